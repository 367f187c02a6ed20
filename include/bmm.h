/* bmm: exact products of packed bit matrices on AMD Instinct MI355X (gfx950).
 *
 * Operations (Karppa & Kaski, "Engineering Boolean Matrix Multiplication for
 * Multiple-Accelerator Shared-Memory Architectures", arXiv 1909.01554):
 *   - the product of an m x k and a k x n bit matrix over the binary field
 *     GF(2) = (0,1,+,*) and over the Boolean algebra (0,1,OR,AND) (section 1;
 *     product definition in section 2.4), by the cubic bit-parallel method
 *     (section 3.18);
 *   - the GF(2) product by the self-inverse alternative-basis Strassen
 *     recursion (Theorem 1, section 2.2; matrix form section 2.8; layers
 *     sections 3.4-3.13): forward basis change of A and B, seven block products
 *     per 2 x 2 level down to a cubic leaf, inverse basis change of C.
 *
 * LAYOUT.  Every matrix is packed row-major in 64-bit words: bit j of row i is
 * bit (j % 64) of word i * ld + j / 64 (least significant bit first).  ld (the
 * row pitch, in words) must be at least ceil(cols / 64).  Bits past the last
 * column of a row (padding) must be zero in A and B; the library writes them
 * as zero in C (with BMM_FLAG_ACCUMULATE it leaves them as they were).
 *
 * MEMORY AND OWNERSHIP.  A, B, C and workspaces are device pointers owned by
 * the caller (for example PyTorch tensors), 8-byte aligned; with
 * BMM_FLAG_HOST_OPERANDS they are page-locked host pointers instead.  A and B
 * are read only.  C must not overlap A, B or the workspace.  The library owns
 * only its internal caches (a transposition scratch buffer per device, plans),
 * released by bmm_finalize().
 *
 * ASYNCHRONY.  Calls enqueue work on `hip_stream` (a hipStream_t; NULL = the
 * default stream) and return without waiting, except where noted.  The return
 * value reports argument and launch errors; faults inside kernels surface at
 * the caller's next synchronization.
 *
 * ERRORS.  Functions return a bmm_status; nothing throws or aborts across this
 * interface.  bmm_last_error() returns a thread-local message for the last
 * failure.
 */
#ifndef BMM_H
#define BMM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  BMM_OK = 0,
  BMM_E_INVAL = -1,       /* bad size, pitch, pointer, alignment or overlap */
  BMM_E_UNSUPPORTED = -2, /* valid request this build cannot do (e.g. Strassen sizes) */
  BMM_E_WORKSPACE = -3,   /* workspace missing or too small */
  BMM_E_NOMEM = -4,       /* a library-owned allocation failed */
  BMM_E_DEVICE = -5       /* a HIP runtime error; message in bmm_last_error() */
} bmm_status;

typedef enum { BMM_GF2 = 0, BMM_BOOLEAN = 1 } bmm_semiring;

/* Leaf kernels for the cubic product. */
typedef enum {
  BMM_LEAF_AUTO = 0,    /* autotuner's choice */
  BMM_LEAF_VALU = 1,    /* bitwise vector ALU leaf (v_bitop3_b32) */
  BMM_LEAF_MFMA_I8 = 2, /* int8 matrix-core leaf, exact int32 counts */
  BMM_LEAF_MFMA_F4 = 3  /* E2M1 (fp4) matrix-core leaf, exact fp32 counts; k < 2^24,
                           else BMM_E_UNSUPPORTED */
} bmm_leaf;

/* 2 x 2 schemes of the GF(2) recursion (bmm_options.scheme). */
typedef enum {
  BMM_SCHEME_SELF_INVERSE = 0, /* alternative basis, Theorem 1 (section 2.2): self-inverse,
                                  in-place basis changes */
  BMM_SCHEME_CHAINING = 1,     /* alternative basis, Theorem 2 (section 2.3): forward and
                                  inverse changes are mutual inverses, so alternative-basis
                                  products chain without changing back in between */
  BMM_SCHEME_WINOGRAD = 2      /* Strassen-Winograd in the standard basis (section 2.1):
                                  no basis changes */
} bmm_scheme;

/* Flags. */
#define BMM_FLAG_ACCUMULATE 0x1u    /* C ^= AB (GF(2)) or C |= AB (Boolean) */
#define BMM_FLAG_B_TRANSPOSED 0x2u  /* B is passed as B^T: n rows of k bits, pitch ldb */
#define BMM_FLAG_ALT_BASIS_IO 0x4u  /* Strassen only: A and B are already in the
                                       alternative basis and C is left in it (the
                                       paper's timing convention, section 4.2) */
#define BMM_FLAG_HOST_OPERANDS 0x8u /* A, B, C are page-locked host memory; blocks
                                       stream through HBM (out-of-core pipeline,
                                       bmm_ooc); the call is then synchronous */
#define BMM_FLAG_OOC_BLOCK_ORDER 0x10u /* out-of-core GF(2): stream the cubic block
                                          order instead of the host-level recursion */
#define BMM_FLAG_LEAN_WORKSPACE 0x40u /* Strassen only: the depth-first levels hold one
                                         child at a time (formed from its parent's
                                         quadrants, its product added into the parent's
                                         result quadrants by gamma) instead of all seven:
                                         their workspace shrinks 7-fold, for more reads
                                         of the parents */
#define BMM_FLAG_INPLACE_BASIS 0x20u /* Strassen only: change A (and B when passed
                                        transposed) to the alternative basis in place
                                        and restore them afterwards, instead of
                                        copying them into the workspace (the basis
                                        changes are invertible in place, section 2.2
                                        and section 3.6) */

typedef struct {
  int leaf;           /* bmm_leaf; 0 = auto */
  int tile;           /* leaf tile variant; -1 or 0 = auto (see bmm_leaf_tiles) */
  int depth_serial;   /* Strassen levels processed one child at a time; -1 = auto */
  int depth_parallel; /* Strassen levels processed breadth-first; -1 = auto */
  int64_t block;      /* out-of-core block size in bits (multiple of 64); 0 = auto */
  uint32_t flags;     /* BMM_FLAG_* */
  int scheme;         /* bmm_scheme of the GF(2) recursion; 0 = self-inverse */
  int shift;          /* Strassen: the last parallel level shifted into the int8 leaf
                         (section 3.15): 0 = off, 1 = on, 2 = on with 8-byte operand
                         loads, -1 = the depth tuner's record for the shape and split
                         (else off).  Applies where the leaf is int8, the scheme is not
                         Winograd, depth_parallel >= 1 and a leaf's k is 2048 or 4096
                         bits; elsewhere the plain leaf runs */
  int64_t k_panel;    /* cubic products (bmm_gf2, bmm_boolean, bmm_cubic_noalloc): k is
                         taken in panels of this many bits (rounded up to whole words),
                         one leaf launch per panel, each panel's product XORed / ORed
                         into C after the first (the sum over j split into consecutive
                         ranges).  Shorter panels keep the operand rows that neighbouring
                         tiles share inside L2 and cut memory traffic, at the price of
                         rereading C once per panel.  0 = the k-panel table's record for
                         the shape (bmm_autotune_k_panel), else one panel; negative = one
                         panel.  Multiples of 128 bits keep 16-byte operand loads */
} bmm_options;

/* Fill *opt with the defaults (everything automatic, no flags). */
void bmm_options_init(bmm_options* opt);

/* Cubic GF(2) product C = AB (or C ^= AB): C[i][k] = XOR_j A[i][j] AND B[j][k].
 * A: m x k (pitch lda), B: k x n (pitch ldb; n x k with BMM_FLAG_B_TRANSPOSED),
 * C: m x n (pitch ldc).  m, k, n >= 0; zero sizes are valid and do nothing
 * (k = 0 writes C = 0 unless accumulating).  Unless B is passed transposed the
 * library transposes it into a cached device scratch buffer (which may call
 * hipMalloc on first use or growth, and synchronizes the device when it grows).
 * That buffer is shared by all such calls on a device, so calls on different
 * streams that may overlap must pass B^T (BMM_FLAG_B_TRANSPOSED).
 * With BMM_FLAG_HOST_OPERANDS, A, B and C are page-locked host memory
 * (hipHostMalloc) and the product runs as bmm_ooc in the cubic block order
 * (opt->block sets the block size): the call waits for earlier work on
 * hip_stream, then returns once C is complete; BMM_FLAG_ACCUMULATE and
 * BMM_FLAG_B_TRANSPOSED are then BMM_E_UNSUPPORTED.
 * Errors: BMM_E_INVAL (negative size, null pointer with nonzero size, pitch too
 * small, C overlapping A or B, host memory not page-locked), BMM_E_NOMEM,
 * BMM_E_DEVICE. */
int bmm_gf2(const uint64_t* A, int64_t lda, const uint64_t* B, int64_t ldb, uint64_t* C,
            int64_t ldc, int64_t m, int64_t k, int64_t n, const bmm_options* opt,
            void* hip_stream);

/* Cubic Boolean product C = AB (or C |= AB): C[i][k] = OR_j A[i][j] AND B[j][k]
 * (section 3.18).  Same arguments and errors as bmm_gf2. */
int bmm_boolean(const uint64_t* A, int64_t lda, const uint64_t* B, int64_t ldb, uint64_t* C,
                int64_t ldc, int64_t m, int64_t k, int64_t n, const bmm_options* opt,
                void* hip_stream);

/* GF(2) product by the 2 x 2 recursion of opt->scheme (default: the
 * self-inverse alternative basis, section 2.2; also the chaining alternative
 * basis, section 2.3, and standard-basis Strassen-Winograd, section 2.1) with
 * `depth` levels of 2 x 2 blocks above a cubic leaf (depth -1 = autotuned;
 * shapes the table lacks take the largest depth whose leaves keep every
 * dimension >= 2048 bits, at most 8; 0 = cubic).
 * Requires m % 2^depth == 0, k % (64 * 2^depth) == 0 and n % (64 * 2^depth) == 0,
 * else BMM_E_UNSUPPORTED.  The workspace (device memory, >= the size from
 * bmm_gf2_strassen_workspace for the same arguments) holds the basis-changed
 * operands and the expanded levels; its contents on return are unspecified.
 * With BMM_FLAG_ALT_BASIS_IO the inputs are taken as A-hat, B-hat and C-hat is
 * returned (no basis changes; B given transposed is then read where it lies).
 * With BMM_FLAG_ACCUMULATE the product is XORed into C (into C-hat under
 * BMM_FLAG_ALT_BASIS_IO; otherwise C is taken to the alternative basis and back).
 * With BMM_FLAG_INPLACE_BASIS the forward change is applied to the caller's A
 * (and to B^T when B is passed transposed; an untransposed B is transposed into
 * the workspace as always) and undone after the product, in stream order: the
 * workspace shrinks by those copies, A and B hold alternative-basis words while
 * the call's work runs (nothing else may read or write them until it finishes),
 * and they hold their original words again once it has.  A and B must not
 * overlap (BMM_E_INVAL).  Should a launch fail midway (BMM_E_DEVICE) their
 * contents are unspecified.
 * With BMM_FLAG_HOST_OPERANDS the operands are page-locked host memory and the
 * product runs as bmm_ooc over GF(2) (host-level recursion levels above the
 * in-HBM recursion; opt->block and opt->depth_* apply, `depth` and the
 * workspace are not used; may be NULL): synchronous as for bmm_gf2;
 * BMM_FLAG_ACCUMULATE, BMM_FLAG_B_TRANSPOSED and BMM_FLAG_ALT_BASIS_IO are then
 * BMM_E_UNSUPPORTED.
 * Errors: as bmm_gf2, plus BMM_E_WORKSPACE. */
int bmm_gf2_strassen(const uint64_t* A, int64_t lda, const uint64_t* B, int64_t ldb,
                     uint64_t* C, int64_t ldc, int64_t m, int64_t k, int64_t n, int depth,
                     void* workspace, size_t workspace_bytes, const bmm_options* opt,
                     void* hip_stream);

/* Workspace bytes that bmm_gf2_strassen needs for these sizes and options
 * (opt->flags matter: BMM_FLAG_ALT_BASIS_IO, BMM_FLAG_INPLACE_BASIS and
 * BMM_FLAG_B_TRANSPOSED decide which operands are staged, BMM_FLAG_LEAN_WORKSPACE how
 * much the depth-first levels hold), and the depth split
 * it will use (either out pointer may be NULL). */
int bmm_gf2_strassen_workspace(int64_t m, int64_t k, int64_t n, int depth,
                               const bmm_options* opt, size_t* bytes_out,
                               int* depth_serial_out, int* depth_parallel_out);

/* One independent product of a batch. */
typedef struct {
  int semiring;           /* bmm_semiring */
  int64_t m, k, n;
  const uint64_t* A;      /* m x k, pitch lda */
  const uint64_t* B;      /* k x n, pitch ldb; or n x k if b_transposed */
  uint64_t* C;            /* m x n, pitch ldc */
  int64_t lda, ldb, ldc;
  int b_transposed;
} bmm_problem;

/* Many independent products of uneven sizes in one persistent launch
 * (workgroups pull work items of 2 x 2 wave tiles from per-XCD device-side
 * queues).  `problems` is a host array, read during the call only.
 * The library keeps a plan per problem table (the pointers, sizes, pitches,
 * semirings and b_transposed flags of every problem, with opt's leaf and tile,
 * on the current device; at most 8, least recently used dropped first, all
 * released by bmm_finalize): the first call with a table allocates its device
 * problem table and a staging buffer for the right operands not given
 * transposed, uploads the table and captures the launch sequence (the
 * transposes into staging, the persistent kernel) into a hipGraph; every call,
 * the first included, then replays that graph on hip_stream and returns without
 * waiting.  The operands' contents are read when the work runs, so a table can
 * be reused with new data in the same buffers.  Calls with the same table are
 * ordered by the library (each waits, on the device, for the previous one, on
 * whatever stream).  Inside stream capture the call enqueues the kernels into
 * the caller's graph; its table's first call must come before, outside the
 * capture (else BMM_E_UNSUPPORTED), and replays of such a graph must not overlap
 * each other or another call with the same table.  New batched tuning records
 * (bmm_autotune_batched, bmm_autotune_load) rebuild the plans on their next use. */
int bmm_batched(const bmm_problem* problems, int64_t count, const bmm_options* opt,
                void* hip_stream);

/* A reusable batched plan: the problem table lives on the device, so a launch
 * is a fixed sequence of kernels that a caller may capture into a hipGraph and
 * replay.  All problems must have b_transposed set.  plan_create allocates
 * device memory (hipMalloc) and synchronizes; plan_launch only enqueues.
 * Launches of one plan share its queue counters: outside stream capture each
 * launch waits (on the device) for the plan's previous one, whatever the
 * stream; launches captured into graphs are not ordered by the library, so
 * replays of those graphs must not overlap each other or other launches of the
 * plan (replay them on one stream). */
int bmm_batched_plan_create(const bmm_problem* problems, int64_t count,
                            const bmm_options* opt, void** plan_out);
int bmm_batched_plan_launch(void* plan, void* hip_stream);
void bmm_batched_plan_destroy(void* plan);
/* Leaf and tile of a batched plan, per problem: opt->leaf and opt->tile where given
 * (BMM_LEAF_MFMA_I8 or BMM_LEAF_MFMA_F4 with tile 1 (128 x 64 output tile per wave),
 * 2 (64 x 64), 3 (64 x 128) or 4 (128 x 64 with the workgroup's operand rows staged
 * through LDS and shared by its four waves); BMM_LEAF_VALU: the VALU leaf, one launch
 * per problem); 0 / AUTO take the autotuner's record for plans of the same problem
 * count and total work (to a factor of two): its choice per size class of k
 * (k < 1024, < 4096, larger) where it recorded one, else its single choice, else int8
 * with tile 4.  Problems with the same matrix-core choice share one persistent launch
 * (workgroups per CU from the same record, else 4); a plan's launch enqueues the VALU
 * products, then each persistent group. */

/* Autotuner for batched plans (the paper's empirical parameter choice,
 * section 3.17, applied to the persistent launch): times one launch of the plan
 * for every matrix-core leaf kind (int8, fp4), tile (1, 2, 3, 4) and persistent grid
 * (2 or 4 workgroups per CU) on the default stream; then, per size class of k, every
 * leaf kind (VALU included) and tile on that class's problems alone, and keeps the
 * per-class choices if the plan they give is faster than the single best choice.
 * Records the result for later plans with AUTO options (saved by bmm_autotune_save)
 * and returns the single best leaf and tile (*seconds_out: the faster of the two
 * plans).  Problems as for bmm_batched_plan_create; their outputs are overwritten.
 * Synchronous; allocates (plans). */
int bmm_autotune_batched(const bmm_problem* problems, int64_t count, int* leaf_out,
                         int* tile_out, double* seconds_out);

/* Out-of-core product of page-locked host matrices (sections 3.3, 3.16, 3.18):
 * C = AB over `semiring` with A, B, C in host memory allocated by hipHostMalloc
 * (else BMM_E_INVAL).  b x b blocks (block bits, a multiple of 64; 0 = option
 * or 2^17) stream through two HBM slots with asynchronous copies on their own
 * streams, overlapped with the leaf; finished C blocks download while the next
 * block computes.  Over GF(2) every block product whose shape admits at least
 * one level runs the alternative-basis recursion in HBM: the uploaded blocks
 * are basis-changed on the device, the products of one C block accumulate in
 * the alternative basis, and the C block changes back once before download
 * (depth_serial = depth_parallel = 0 in opt forces the cubic leaf).
 * Synchronous: returns after C is complete; *seconds_out (if not NULL)
 * receives the wall time.  Allocates and frees its HBM buffers. */
int bmm_ooc(int semiring, const uint64_t* A, int64_t lda, const uint64_t* B, int64_t ldb,
            uint64_t* C, int64_t ldc, int64_t m, int64_t k, int64_t n, int64_t block,
            const bmm_options* opt, double* seconds_out);

/* Host <-> device transfers of the calling thread's last successful bmm_ooc call
 * (also when reached through BMM_FLAG_HOST_OPERANDS), per direction: bytes moved
 * and the summed durations of the copies themselves (HIP events around each copy
 * on its own stream), so bytes / seconds is the PCIe rate while data moves.  Any
 * pointer may be NULL; zeros before the first call. */
int bmm_ooc_last_transfers(double* h2d_bytes, double* h2d_seconds, double* d2h_bytes,
                           double* d2h_seconds);

/* Stage entry points of the recursion (for kernel-by-kernel checks and for
 * callers that build their own schedules).  All enqueue on hip_stream.
 *
 * bmm_transpose: dst (cols x rows bits, pitch ldd) = src^T (src rows x cols bits). */
int bmm_transpose(const uint64_t* src, int64_t lds, uint64_t* dst, int64_t ldd, int64_t rows,
                  int64_t cols, void* hip_stream);
/* bmm_basis_change: in place on a rows x (64 * row_words) matrix, the 2 x 2
 * basis change of `scheme` (bmm_scheme) at the top `depth` levels: inverse = 0
 * applies the forward change (eq. mb-fwdbasisrecurrence for the self-inverse
 * design, eq. ab-fwdbasisrecurrence for chaining), 1 the inverse change of the
 * result (eqs. mb-revbasisrecurrence, ab-revbasisrecurrence).  transposed = 1:
 * X is a right-hand operand stored transposed (its 01 and 10 quadrants trade
 * places at every level).  The Winograd scheme has no basis change (no-op).
 * rows and row_words must be divisible by 2^depth. */
int bmm_basis_change(uint64_t* X, int64_t ld, int64_t rows, int64_t row_words, int depth,
                     int inverse, int scheme, int transposed, void* hip_stream);
/* bmm_expand: one level (levels = 1) or two merged levels (levels = 2) of the
 * operand linear combinations of `scheme` (eqs. mb-tsrecurrence,
 * ab-tsrecurrence, sw-input) for `parents` matrices of rows x (64 * words)
 * (parent p at src + p * strideP, pitch ldp).  side 0 = left operand (alpha),
 * 1 = right operand stored transposed (beta).  Children are written compactly
 * to dst: 7^levels per parent, in order. */
int bmm_expand(int side, int levels, int scheme, const uint64_t* src, int64_t ldp,
               int64_t strideP, uint64_t* dst, int64_t rows, int64_t words, int64_t parents,
               void* hip_stream);
/* bmm_compress: the combination of products of `scheme` (eqs. mb-qrecurrence,
 * ab-qrecurrence, sw-output): 7^levels compact children per parent combine
 * into the parents' quadrants. */
int bmm_compress(int levels, int scheme, const uint64_t* src, uint64_t* dst, int64_t ldp,
                 int64_t strideP, int64_t rows, int64_t words, int64_t parents,
                 void* hip_stream);

/* Number of tile variants of a leaf (valid values of bmm_options.tile are
 * 1..count; 0 = auto), and the C tile (rows x columns) of a variant (per workgroup for
 * the VALU leaf, per wave for the matrix-core leaves).  The VALU leaf's tile 1 is the
 * dot-product form against B^T (128 x 128); tile 2 is the outer-product form (512 x
 * 1024): each bit of A selects a row of B, whose words the waves read from LDS at one
 * address per wave, and the accumulators are the result bits.  Tile 2 reads B row-major, so it
 * serves the cubic products only (a B passed transposed is transposed back into
 * scratch first); batched leaves (the recursion, bmm_batched) given VALU tile 2 run
 * tile 1. */
int bmm_leaf_tiles(int leaf, int* count_out);
int bmm_leaf_tile_shape(int leaf, int tile, int* rows_out, int* cols_out);
/* The leaf kind and tile a cubic product (batch = 1) or a batch of equal leaf
 * products of this shape would run with these options (the autotune table's
 * entry, else the default rule); no device work. */
int bmm_leaf_choice(int semiring, int64_t m, int64_t k, int64_t n, int64_t batch,
                    const bmm_options* opt, int* leaf_out, int* tile_out);

/* Autotuner (the paper fixes its layer depths empirically under memory limits,
 * section 3.17).  Leaf table: bmm_autotune_leaf times every leaf kernel and tile
 * on `batch` independent m x k x n products (batch bucketed to 1, 2, 4, ..., 64;
 * allocates and frees scratch, synchronizes) and records the fastest for
 * BMM_LEAF_AUTO / tile 0; bmm_autotune_cubic is the batch-1 case;
 * bmm_autotune_set records an entry by hand.  Depth table:
 * bmm_autotune_strassen times bmm_gf2_strassen on the caller's operands for the
 * deepest four admissible depths (leaves >= 1024 bits), each with the plain leaf
 * and, where it applies, with the last level shifted into the leaf (shift 1 and 2),
 * each with the fewest depth-first levels whose workspace fits, and records the
 * fastest (depth, split, shift) for depth -1.
 * The tables (these two, the k-panel table below and the batched plans' records) are
 * per process and can be saved to / loaded from a text file. */
int bmm_autotune_leaf(int semiring, int64_t m, int64_t k, int64_t n, int64_t batch,
                      int* leaf_out, int* tile_out, double* seconds_out);
int bmm_autotune_cubic(int semiring, int64_t m, int64_t k, int64_t n, int* leaf_out,
                       int* tile_out, double* seconds_out);
int bmm_autotune_set(int semiring, int64_t m, int64_t k, int64_t n, int64_t batch, int leaf,
                     int tile);
int bmm_autotune_strassen(const uint64_t* A, int64_t lda, const uint64_t* B, int64_t ldb,
                          uint64_t* C, int64_t ldc, int64_t m, int64_t k, int64_t n,
                          void* workspace, size_t workspace_bytes, const bmm_options* opt,
                          int* depth_out, int* depth_serial_out, int* shift_out,
                          double* seconds_out);
/* k-panel table: times bmm_gf2 / bmm_boolean on the caller's device operands (B as
 * opt->flags say; BMM_FLAG_ACCUMULATE and BMM_FLAG_HOST_OPERANDS are BMM_E_INVAL)
 * with each candidate panel length (candidates[0..count-1] in bits; count 0: one
 * panel and every power of two from 8192 below k), once after one warm-up, and
 * records the fastest for k_panel = 0.  The result depends on the operands' bits
 * (dense operands draw more power, which the shorter panels' lower memory traffic
 * relieves), so tune on representative data.  C holds the product on return. */
int bmm_autotune_k_panel(int semiring, const uint64_t* A, int64_t lda, const uint64_t* B,
                         int64_t ldb, uint64_t* C, int64_t ldc, int64_t m, int64_t k, int64_t n,
                         const bmm_options* opt, const int64_t* candidates, int count,
                         int64_t* panel_out, double* seconds_out);
int bmm_autotune_save(const char* path);
int bmm_autotune_load(const char* path);

/* VALU roofline calibration (the bit-operation peak of section 1.2 is a device's
 * lane-operation rate times its word width; this measures that rate for the
 * three-input v_bitop3_b32 that the VALU leaf folds with, instead of assuming
 * it).  waves_per_simd (1..8) waves on every SIMD of every CU each fold 16
 * independent 32-bit chains, one v_bitop3_b32 per chain per round, for `rounds`
 * rounds (a positive multiple of 4), with no memory traffic in the timed loop;
 * every wave reads the core-clock counter (s_memtime) and the constant-rate
 * counter before and after.  Outputs (any may be NULL):
 *   lane_ops_per_clk_cu: all waves' lane operations (64 per instruction) over the
 *                        launch's core cycles (HIP-event time x clock_ghz) and the
 *                        CU count;
 *   clock_ghz:           median core clock of the waves;
 *   seconds:             the timed launch by HIP events;
 *   aggregate_bops:      2 x 32 bit operations per lane operation, all waves,
 *                        over `seconds`.
 * Synchronous on the default stream; allocates a few MiB. */
int bmm_calibrate_valu(int waves_per_simd, int64_t rounds, double* lane_ops_per_clk_cu,
                       double* clock_ghz, double* seconds, double* aggregate_bops);

/* Cubic product that allocates nothing, for callers that cannot call hipMalloc
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * allocation).  Same operation, arguments and errors as bmm_gf2 (semiring =
 * BMM_GF2) and bmm_boolean (BMM_BOOLEAN), and the same kernels; when B is not
 * passed transposed, B^T is staged in a fixed device array of
 * BMM_NOALLOC_SCRATCH_BYTES instead of the library's growable buffer, so
 * n * ceil(k / 64) * 8 must not exceed that size (else BMM_E_UNSUPPORTED; pass
 * BMM_FLAG_B_TRANSPOSED to use no scratch at all).  Each device holds its own
 * copy of the array from the first call on it until the process ends; that
 * first call looks up its address (hipGetSymbolAddress), later ones touch no
 * runtime state.  All calls on one device share the array: two such calls that
 * may overlap on one device (different streams, or a graph replayed on one
 * stream while another call runs on a second) race on it and must be ordered
 * by the caller.  BMM_FLAG_HOST_OPERANDS is refused (BMM_E_UNSUPPORTED). */
#define BMM_NOALLOC_SCRATCH_BYTES (32u << 20)
int bmm_cubic_noalloc(int semiring, const uint64_t* A, int64_t lda, const uint64_t* B,
                      int64_t ldb, uint64_t* C, int64_t ldc, int64_t m, int64_t k, int64_t n,
                      const bmm_options* opt, void* hip_stream);

/* Testing hook: the next `count` device allocations the library makes (scratch,
 * plans, staging, out-of-core buffers, autotuner buffers) fail as if the device
 * were out of memory, so callers' error paths can be exercised; the entry point
 * then returns BMM_E_NOMEM and leaves no allocation behind.  count <= 0 disarms.
 * Process-wide. */
int bmm_debug_fail_allocations(int64_t count);

const char* bmm_status_string(int status);
const char* bmm_last_error(void);
const char* bmm_version(void);
/* Free library-owned device memory (scratch, plans' caches).  Not thread-safe
 * against concurrent calls on other threads. */
void bmm_finalize(void);

#ifdef __cplusplus
}
#endif

#endif /* BMM_H */
