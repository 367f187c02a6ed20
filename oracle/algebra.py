"""The paper's 2x2 block algorithms as straight-line programs (section 2).

TEST INFRASTRUCTURE ONLY (part of the oracle).

Each program works on any block type that supports ``^`` (XOR over GF(2)):
numpy arrays of bits or of packed words, Python ints, or counting stand-ins.
Block index order is (00, 01, 10, 11); the seven products are numbered 0..6.

* Self-inverse alternative basis (Theorem 1, section 2.2): forward basis
  change eq. mb-fwdbasisrecurrence, linear combinations eq. mb-tsrecurrence,
  product combination eq. mb-qrecurrence, inverse basis change
  eq. mb-revbasisrecurrence.
* Chaining alternative basis (Theorem 2, section 2.3): eqs. ab-fwdbasisrecurrence,
  ab-revbasisrecurrence, ab-tsrecurrence, ab-qrecurrence.
* Strassen-Winograd in the standard basis (section 2.1): eqs. sw-input,
  sw-output.

``matrix_of`` derives a program's GF(2) matrix by feeding it unit vectors, so
the tests can compare these programs with the matrices printed in section 2.8.
"""
import itertools

import numpy as np


# ---- Theorem 1: self-inverse, in-place basis changes (section 2.2) ----

def sinv_fwd(X00, X01, X10, X11):
    """eq. mb-fwdbasisrecurrence: only the 11 block changes, to X01 + X10 + X11."""
    return X00, X01, X10, X01 ^ X10 ^ X11


def sinv_alpha(A00, A01, A10, A11):
    """eq. mb-tsrecurrence, left operand."""
    return A00, A01, A10, A11, A00 ^ A11, A01 ^ A11, A10 ^ A11


def sinv_beta(B00, B01, B10, B11):
    """eq. mb-tsrecurrence, right operand."""
    return B00, B10, B00 ^ B11, B11, B01, B01 ^ B11, B10 ^ B11


def sinv_gamma(Q0, Q1, Q2, Q3, Q4, Q5, Q6):
    """eq. mb-qrecurrence."""
    return Q0 ^ Q1, Q4 ^ Q6, Q2 ^ Q5, Q1 ^ Q3 ^ Q5 ^ Q6


def sinv_inv(C00, C01, C10, C11):
    """eq. mb-revbasisrecurrence: the 01 and 10 blocks gain the 11 block."""
    return C00, C01 ^ C11, C10 ^ C11, C11


# ---- Theorem 2: chaining (section 2.3) ----

def chain_fwd(X00, X01, X10, X11):
    """eq. ab-fwdbasisrecurrence (the 11 block is formed first, then the 10 block)."""
    h11 = X01 ^ X11
    h10 = h11 ^ X10
    return X00, X01, h10, h11


def chain_inv(H00, H01, H10, H11):
    """eq. ab-revbasisrecurrence."""
    return H00, H01, H10 ^ H11, H01 ^ H11


def chain_alpha(A00, A01, A10, A11):
    """eq. ab-tsrecurrence, left operand."""
    return A00, A01, A10, A11, A00 ^ A10, A01 ^ A10, A10 ^ A11


def chain_beta(B00, B01, B10, B11):
    """eq. ab-tsrecurrence, right operand."""
    return B00, B10 ^ B11, B10, B11, B01, B01 ^ B10, B00 ^ B10


def chain_gamma(Q0, Q1, Q2, Q3, Q4, Q5, Q6):
    """eq. ab-qrecurrence (R is the shared partial sum)."""
    R = Q1 ^ Q2 ^ Q4
    return Q0 ^ Q1, R ^ Q5, R ^ Q6, Q3 ^ Q4


# ---- Strassen-Winograd, standard basis (section 2.1) ----

def sw_xi(A00, A01, A10, A11):
    """eq. sw-input, left operand (T2 feeds T3, T3 feeds T4)."""
    T0 = A10 ^ A11
    T1 = A01
    T2 = A01 ^ A11
    T3 = A10 ^ T2
    T4 = A00 ^ T3
    return T0, T1, T2, T3, T4, A10, A00


def sw_eta(B00, B01, B10, B11):
    """eq. sw-input, right operand."""
    S0 = B10 ^ B11
    S1 = B10
    S2 = B01 ^ B11
    S3 = B10 ^ S2
    S4 = B01
    S5 = B00 ^ S3
    return S0, S1, S2, S3, S4, S5, B00


def sw_zeta(Q0, Q1, Q2, Q3, Q4, Q5, Q6):
    """eq. sw-output."""
    U0 = Q1 ^ Q3
    U1 = Q2 ^ U0
    U2 = Q4 ^ U0
    return Q1 ^ Q6, Q0 ^ U2, Q5 ^ U1, Q0 ^ U1


class Decomposition:
    """One 2x2 scheme: basis changes (fwd for both operands, inv for the
    result) and the linear maps alpha, beta, gamma."""

    def __init__(self, name, fwd, alpha, beta, gamma, inv):
        self.name = name
        self.fwd = fwd
        self.alpha = alpha
        self.beta = beta
        self.gamma = gamma
        self.inv = inv


def _identity4(*x):
    return tuple(x)


SELF_INVERSE = Decomposition("self-inverse", sinv_fwd, sinv_alpha, sinv_beta, sinv_gamma,
                             sinv_inv)
CHAINING = Decomposition("chaining", chain_fwd, chain_alpha, chain_beta, chain_gamma,
                         chain_inv)
STRASSEN_WINOGRAD = Decomposition("strassen-winograd", _identity4, sw_xi, sw_eta, sw_zeta,
                                  _identity4)


def matrix_of(prog, n_in):
    """The GF(2) matrix (outputs x inputs) that a linear straight-line program computes."""
    cols = []
    for c in range(n_in):
        e = [0] * n_in
        e[c] = 1
        cols.append([int(v) & 1 for v in prog(*e)])
    return np.array(cols, dtype=np.int64).T


class Counted:
    """A block stand-in that counts bit additions: XOR of two blocks of
    `size` bits costs `size` bit operations."""

    counter = [0]

    def __init__(self, size):
        self.size = size

    def __xor__(self, other):
        assert self.size == other.size
        Counted.counter[0] += self.size
        return Counted(self.size)


def slp_additions(prog, n_in):
    """Number of additions a straight-line program performs on unit-size blocks."""
    Counted.counter[0] = 0
    prog(*[Counted(1) for _ in range(n_in)])
    return Counted.counter[0]


def triple_product_ok(zeta, xi, eta, s=2, t=2, u=2):
    """eq. triple-prod: sum_h zeta[i'k',h] xi[h,ij] eta[h,j'k] = [i=i'][j=j'][k=k'] over GF(2)."""
    r = xi.shape[0]
    for i, ip, j, jp, k, kp in itertools.product(range(s), range(s), range(t), range(t),
                                                 range(u), range(u)):
        acc = 0
        for h in range(r):
            acc ^= int(zeta[ip * u + kp, h]) & int(xi[h, i * t + j]) & int(eta[h, jp * u + k])
        want = int(i == ip and j == jp and k == kp)
        if acc != want:
            return False
    return True
