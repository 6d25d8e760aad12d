/*
 * ozaki.h - emulated-FP64 (Ozaki scheme) GEMM, two-site H_eff.psi and a
 * Davidson eigensolver step on AMD Instinct MI355X (gfx950).
 *
 * Method (arXiv 2510.04795, "Theory of emulated FP64 arithmetic"): for
 * C = A B, (1) convert A and B to fixed point with one power-of-two exponent
 * per row of A and per column of B, (2) split both into S int8 slices,
 * (3) multiply slice pairs exactly in low precision (int8 MFMA, int32
 * accumulation), (4) accumulate the pair products and convert back to FP64.
 * The slice count follows "Numerical procedure": S slices carry 8S - 1
 * mantissa bits plus the sign, S = ceildiv(bits + 1, 8).
 *
 * Conventions shared by every entry point
 *  - Matrices are FP64, row-major, with a leading dimension (elements).
 *    Matrix and vector pointers are DEVICE pointers owned by the caller
 *    unless stated otherwise.
 *  - stream is a hipStream_t passed as void* (NULL = the null stream).
 *    Enqueue calls (ozaki_dgemm, heff_apply) are asynchronous, allocate
 *    nothing and never synchronise, so they can be captured in a hipGraph.
 *    *_create calls may allocate and synchronise; *_destroy frees what the
 *    matching *_create allocated.
 *  - Every call returns an int status (OZ_*): 0 success, > 0 informational,
 *    < 0 error.  No exception crosses this interface.  The text of the last
 *    error raised on the calling host thread is ozaki_last_error().
 *  - An ozaki_ctx (and every plan made from it) is bound to one device and
 *    must be used by one host thread at a time.
 *  - Emulated arithmetic: S = slices in [2, 8]; G = ndiag diagonals of the
 *    S x S slice-pair grid are kept (pairs with s + t < G).  ndiag = 0 means
 *    G = S (drop the less significant lower triangle); the accepted values
 *    are G in {S, S + 1, 2S - 1} (2S - 1 keeps all S^2 pairs).  slices = 0
 *    selects the native FP64 MFMA path where an entry point offers it.
 *  - Results of the emulated path are deterministic and independent of the
 *    launch configuration: integer pair products are exact, the FP64
 *    recombination runs in one fixed order per output element.
 *  - A row of op(A) or a column of op(B) that holds a NaN or an Inf makes
 *    the matching row / column of the result NaN and sets the sticky
 *    OZ_FLAG_NONFINITE bit of the context (ozaki_ctx_flags).
 */
#ifndef OZAKI_H
#define OZAKI_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ---------------------------------------------------- */
#define OZ_OK 0
#define OZ_CONVERGED 1        /* davidson_step: residual norm <= tol          */
#define OZ_STAGNATED 2        /* davidson_step: residual stopped decreasing   */
#define OZ_MAX_ITER 3         /* davidson_step: iteration limit reached       */
#define OZ_ERR_ARG (-1)       /* invalid argument (message in ozaki_last_error) */
#define OZ_ERR_WORKSPACE (-2) /* workspace missing or too small               */
#define OZ_ERR_HIP (-3)       /* HIP runtime error (no device, launch failure) */
#define OZ_ERR_UNSUPPORTED (-4) /* valid request this library does not provide*/
#define OZ_ERR_STATE (-5)     /* object used in the wrong state               */
#define OZ_ERR_NOMEM (-6)     /* device or host allocation failed             */

#define OZ_FLAG_NONFINITE 1u  /* some input row/column held NaN or Inf        */

/* Exponent reported by ozaki_split for a row/column holding NaN or Inf. */
#define OZ_EXP_NONFINITE INT32_MIN

typedef struct ozaki_ctx_s *ozaki_ctx;
typedef struct heff_plan_s *heff_plan;
typedef struct davidson_s *davidson;

/* Text for a status code (static storage). */
const char *ozaki_status_string(int status);
/* Text of the last error on this host thread ("" if none). */
const char *ozaki_last_error(void);
/* Library version as major * 10000 + minor * 100 + patch. */
int ozaki_version(void);

/* ---- context --------------------------------------------------------- */
/* Bind a context to HIP device `device`.  Allocates a 4-byte flag word on
 * that device.  OZ_ERR_HIP when the device does not exist. */
int ozaki_ctx_create(ozaki_ctx *out, int device);
int ozaki_ctx_destroy(ozaki_ctx ctx);
/* Read and clear the sticky flags (synchronises the device). */
int ozaki_ctx_flags(ozaki_ctx ctx, uint32_t *flags_out);

/* Per-phase timing for benchmarks.  With timing enabled, the enqueue calls
 * record a hipEvent pair on their stream around each phase (at most 4096
 * phases are kept); ozaki_ctx_phase_times waits for the recorded events and
 * returns how many phases it wrote, phase[i] = OZ_PHASE_* and ms[i] = the
 * elapsed milliseconds, then clears the record.  Enabling allocates events
 * (do not enable during graph capture). */
#define OZ_PHASE_SLICE 1      /* exponents + int8 slices of GEMM operands     */
#define OZ_PHASE_PAIR 2       /* int8 pair GEMM + FP64 recombination          */
#define OZ_PHASE_FP64 3       /* native FP64 MFMA GEMM                        */
#define OZ_PHASE_HEFF_L 4     /* H_eff.psi first contraction (all operators)  */
#define OZ_PHASE_HEFF_R 5     /* H_eff.psi second contraction + accumulation  */
#define OZ_PHASE_HEFF_AUX 6   /* H_eff.psi slicing of psi / T and diagonal    */
int ozaki_ctx_set_timing(ozaki_ctx ctx, int enable);
int ozaki_ctx_phase_times(ozaki_ctx ctx, int32_t *phase, double *ms, int32_t max_phases);

/* ---- parameters ------------------------------------------------------ */
/* S = ceildiv(mantissa_bits + 1, 8) ("Numerical procedure"); OZ_ERR_ARG if
 * bits < 1. */
int ozaki_slices_for_bits(int mantissa_bits);
/* Number of slice pairs (s, t) with s + t < ndiag (0 -> S); the worked
 * example of the paper's four-step strategy has 7 x 7 = 49 in full mode.
 * < 0 for invalid arguments. */
int ozaki_pair_count(int slices, int ndiag);
/* Largest inner dimension whose int32 diagonal sums cannot overflow
 * (every product is at most 2^14 in magnitude); above it ozaki_dgemm
 * accumulates K-chunks in int64 workspace, with an identical result. */
int64_t ozaki_max_exact_k(int slices, int ndiag);

/* ---- emulated / native DGEMM ---------------------------------------- */
/* Workspace (bytes) ozaki_dgemm needs for this problem (0 for slices = 0).
 * Holds the int8 slices of op(A) and op(B) with their exponents, plus int64
 * partial sums when K > ozaki_max_exact_k. */
size_t ozaki_dgemm_workspace_bytes(int64_t M, int64_t N, int64_t K, int slices, int ndiag);

/* C = alpha op(A) op(B) + beta C   ("Theory of emulated FP64 arithmetic").
 *  transa/transb 'N' or 'T' (row-major BLAS meaning: op(A) is M x K);
 *  beta == 0: C is not read (may hold NaN);
 *  slices in [2, 8] (emulated) or 0 (native FP64 MFMA GEMM);
 *  the emulated output element is
 *     h = Q_{G-1}; h = h * 2^-8 + Q_g (g = G-2 .. 0), c = h * 2^(e_i + f_j - 14),
 *     C = alpha * c (beta == 0) or fma(alpha, c, beta * C),
 *  with Q_g the exact int sum of slice pairs on diagonal g, e_i / f_j the
 *  shared exponents of row i of op(A) and column j of op(B).
 *  workspace: device memory of at least ozaki_dgemm_workspace_bytes, 256-byte
 *  aligned; it may be NULL when that size is 0.  Errors: OZ_ERR_ARG (bad
 *  sizes, lda/ldb/ldc, trans, slices, ndiag), OZ_ERR_WORKSPACE, OZ_ERR_HIP. */
int ozaki_dgemm(ozaki_ctx ctx, char transa, char transb, int64_t M, int64_t N, int64_t K,
                double alpha, const double *A, int64_t lda, const double *B, int64_t ldb,
                double beta, double *C, int64_t ldc, int slices, int ndiag,
                void *workspace, size_t workspace_bytes, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc):
 * ozaki_dgemm with the same arguments, arithmetic and results, whose
 * workspace is a library-held device buffer of OZ_STATIC_WORKSPACE_BYTES on
 * each GPU (held from the library's load on that GPU until the process
 * ends; its address is looked up by ozaki_ctx_create).  The call allocates
 * nothing and does not synchronise.  Products that need more workspace than
 * that (ozaki_dgemm_workspace_bytes; e.g. square n = 2048 needs 57 MiB at
 * S = 7 and 64 MiB at S = 8) fail with OZ_ERR_WORKSPACE before anything is
 * launched.  Nothing in the buffer must start at zero: every call writes
 * what it reads.  All calls on one GPU share the buffer, so calls whose
 * execution overlaps on one GPU (other streams, other host threads) race:
 * order them, e.g. issue them on one stream.  Errors as ozaki_dgemm. */
#define OZ_STATIC_WORKSPACE_BYTES (96ull << 20)
int ozaki_dgemm_static(ozaki_ctx ctx, char transa, char transb, int64_t M, int64_t N, int64_t K,
                       double alpha, const double *A, int64_t lda, const double *B, int64_t ldb,
                       double beta, double *C, int64_t ldc, int slices, int ndiag, void *stream);

/* ---- emulation modes: mantissa width, automatic width, dispatch ------ */
/* The paper's library lets the user give the mantissa width, or finds the
 * width that keeps native FP64 accuracy itself, and uses emulation eagerly
 * or only where it is faster ("Numerical procedure"; the rules there belong
 * to a vendor library and are not published).  This library's rules:
 *
 * ozaki_choose_slices: statistics of the operands (one exponent pass and one
 *  sum-of-squares pass over each, copied to the host: synchronises `stream`)
 *  give rho_A = root mean square over the rows i of op(A) of
 *  2^e_i / rms(row i), and rho_B over the columns of op(B).  Predicted
 *  relative Frobenius errors:
 *    emulated(S, G) = 0.75 2^-8S [ (rho_A + rho_B) / sqrt(3)
 *                               + sqrt(n_G) (65536 / 12 / 2^14) rho_A rho_B 2^-8(G-S) ]
 *    native(K)      = 0.3 2^-53 sqrt(K)
 *  (n_G: slice pairs on the first dropped diagonal; the factors 0.75 and
 *  0.3 fitted to measured errors).  Chosen: the (S, G), S in [2, 8],
 *  G in {S, S + 1}, with the fewest slice pairs whose prediction is no larger
 *  than native(K); (8, 9) if none; (2, 2) if an operand is all zeros; (7, 7)
 *  if an operand holds NaN/Inf.
 *  stats_out (nullable, host, 4 doubles): rho_A, rho_B, emulated(S, G),
 *  native(K).  workspace: ozaki_dgemm_auto_workspace_bytes(M, N, K) bytes. */
int ozaki_choose_slices(ozaki_ctx ctx, char transa, char transb, int64_t M, int64_t N, int64_t K,
                        const double *A, int64_t lda, const double *B, int64_t ldb, void *workspace,
                        size_t workspace_bytes, void *stream, int32_t *slices_out, int32_t *ndiag_out,
                        double *stats_out);
/* Workspace of ozaki_dgemm_auto and ozaki_choose_slices (covers every (S, G)
 * the automatic choice can return). */
size_t ozaki_dgemm_auto_workspace_bytes(int64_t M, int64_t N, int64_t K);
/* C = alpha op(A) op(B) + beta C with the width and path chosen here:
 *  bits > 0: S = ozaki_slices_for_bits(bits) clamped to [2, 8], ndiag = S;
 *  bits = 0: (S, G) from ozaki_choose_slices (synchronises).
 *  performant = 0 (eager): the emulated GEMM with that (S, G).
 *  performant = 1: the first call of a (transa, transb, M, N, K, S, G) with
 *   beta = 0 runs the native FP64 and the emulated GEMM once each into C,
 *   timed (synchronises), keeps the faster for this context and then computes
 *   C with it; later calls of that shape use the kept path; a shape not yet
 *   timed (first seen with beta != 0) uses the emulated path.
 *  slices_out, ndiag_out (nullable, host): the path taken (0, 0: native FP64).
 *  Results are those of ozaki_dgemm with that (slices, ndiag).  Errors as for
 *  ozaki_dgemm; OZ_ERR_ARG for bits < 0 or performant not 0 / 1. */
int ozaki_dgemm_auto(ozaki_ctx ctx, char transa, char transb, int64_t M, int64_t N, int64_t K,
                     double alpha, const double *A, int64_t lda, const double *B, int64_t ldb,
                     double beta, double *C, int64_t ldc, int bits, int performant, void *workspace,
                     size_t workspace_bytes, void *stream, int32_t *slices_out, int32_t *ndiag_out);

/* ---- tile variants and autotuning ------------------------------------ */
/* The int8 pair GEMM is built in several tile variants per (S, G) (waves of
 * MB x NB blocks of 32 x 32 outputs).  Every variant gives bit-identical
 * results; only speed differs.  ozaki_pair_variants writes the tile shape of
 * variant v to tile_m[v] x tile_n[v] (0 x 0 when v is not built for this G)
 * and returns the number of variant slots. */
int ozaki_pair_variants(int slices, int ndiag, int32_t *tile_m, int32_t *tile_n, int32_t max_variants);
/* Use variant `variant` for (slices, ndiag) in this context (-1: library
 * default; heff plans then autotune if enabled).  OZ_ERR_ARG for a variant
 * that is not built. */
int ozaki_ctx_set_variant(ozaki_ctx ctx, int slices, int ndiag, int variant);
/* Variant ozaki_dgemm currently uses for (slices, ndiag). */
int ozaki_ctx_get_variant(ozaki_ctx ctx, int slices, int ndiag);
/* Whether heff_plan_create times the variants of its two grouped phases and
 * keeps the fastest (default on; a variant fixed with ozaki_ctx_set_variant
 * takes precedence). */
int ozaki_ctx_set_autotune(ozaki_ctx ctx, int enable);
/* Launch codes of the resident kernel (first phase) and of the
 * paired-term kernel (second phase) (ozaki_ctx_set_heff_launch,
 * ozaki_ctx_set_heff_phase, heff_plan_phase). */
#define OZ_HEFF_LAUNCH_RESIDENT (-2)
#define OZ_HEFF_LAUNCH_PAIRED_TERMS (-3)
/* How heff plans created afterwards launch their two grouped pair phases:
 * 0 = one workgroup per output tile; k > 0 = the streamed kernel, in which
 * as many workgroups as fit at once on min(k, number of CUs) compute units
 * walk the tile list and the first K block of each (tile, term) item is
 * loaded during the last block of the item before it;
 * OZ_HEFF_LAUNCH_RESIDENT = the first phase on the resident kernel where it
 * is built for the tile variant (one 32 x 32 block per wave on the
 * three-stage LDS ring), the second one workgroup per tile: a grid that
 * fits on the device at once, each workgroup walking its part of a
 * schedule the plan balances by cost, the K blocks of its consecutive tiles
 * streamed through one ring (a tile's first blocks load during the
 * previous tile's last blocks and epilogue); OZ_HEFF_LAUNCH_PAIRED_TERMS =
 * the first phase one workgroup per tile, the second on the paired-term
 * kernel where it is built (64 x 64 tiles of variant 0 with the
 * three-stage ring, S <= 6): eight waves per tile in two groups with a
 * ring each, taking the tile's terms two at a time and adding their FP64
 * values in term order (for outputs too small to give every SIMD two
 * waves otherwise); -1 (default) = when autotuning is on, time the first
 * phase one workgroup per tile, streamed (if its items average at most 16
 * K blocks) and resident (where built), the second one workgroup per tile
 * and paired (where built); else 0.  Results are bit-identical in every
 * mode.  OZ_ERR_ARG for mode < -3. */
int ozaki_ctx_set_heff_launch(ozaki_ctx ctx, int mode);
/* Device bytes that heff plans created afterwards may use for the
 * intermediates T_u = L psi of the first products (FP64 values, and their
 * slices and exponents when emulated); 0 (default) = 8 GiB.  A plan cuts its
 * triple list into contiguous chunks whose distinct first products fit
 * (always at least one triple per chunk) and runs them in order within each
 * apply; sigma tiles continue across chunks from their stored values, so
 * the result is bit-identical for every budget. */
int ozaki_ctx_set_heff_budget(ozaki_ctx ctx, size_t bytes);
/* Fix the choice of one grouped phase (0 = first product, 1 = second) for
 * emulated heff plans created afterwards: tile variant (see
 * ozaki_pair_variants; < 0 clears the fix), tile order (0 = cost-balanced
 * contiguous parts per XCD, 1 = longest tile first, 2 = whole outputs to
 * the least loaded XCD, heaviest first) and launch (0 = one
 * workgroup per tile, k > 0 = streamed on k compute units,
 * OZ_HEFF_LAUNCH_RESIDENT = the resident kernel, first phase only,
 * OZ_HEFF_LAUNCH_PAIRED_TERMS = the paired-term kernel, second phase
 * only).  With both
 * phases fixed a plan times nothing, which reproduces a timed plan's choice
 * (heff_plan_phase) exactly, e.g. for profiling.  OZ_ERR_ARG for an unknown
 * phase, variant, order or launch; a variant not built for the plan's
 * (S, G), or a resident or paired-term launch not built for it or asked
 * for the other phase, makes heff_plan_create fail with OZ_ERR_ARG. */
int ozaki_ctx_set_heff_phase(ozaki_ctx ctx, int phase, int variant, int order, int launch);
/* Time every built variant of this GEMM (alpha = 1, beta = 0 into C, one
 * warm-up and three timed calls each) and fix the fastest for (slices,
 * ndiag) in the context.  ms_out (host, nullable, one slot per variant) gets
 * the mean milliseconds or -1.  Returns the chosen variant (>= 0) or an
 * error; synchronises the stream. */
int ozaki_dgemm_tune(ozaki_ctx ctx, char transa, char transb, int64_t M, int64_t N, int64_t K,
                     const double *A, int64_t lda, const double *B, int64_t ldb, double *C,
                     int64_t ldc, int slices, int ndiag, void *workspace, size_t workspace_bytes,
                     void *stream, double *ms_out);

/* ---- test and debug surface (steps 1-3 on their own) ---------------- */
/* Steps 1-2: shared exponents and slices of X (rows x cols, row-major, ld).
 *  by_columns = 0: one exponent per row, digits[S][rows][cols];
 *  by_columns = 1: one exponent per column, digits[S][cols][rows] (each
 *  column's digits contiguous, as the B operand is consumed).
 *  Digits are balanced base 256 (most significant slice first):
 *  RNE(x 2^(8S-1-e)) = sum_t d_t 256^(S-1-t), d_t in [-128, 127].
 *  exps gets e per group, OZ_EXP_NONFINITE for a group holding NaN/Inf (its
 *  digits are 0).  Uses context-owned scratch (may allocate; not for graph
 *  capture).  Synchronises the stream before returning. */
int ozaki_split(ozaki_ctx ctx, int by_columns, int64_t rows, int64_t cols, const double *X,
                int64_t ld, int slices, int8_t *digits, int32_t *exps, void *stream);
/* Step 3: Q[g][i][j] = sum over kept pairs (s + t = g) and k of
 * Adig[s][i][k] * BTdig[t][j][k], g < G, as int32 (exact for
 * K <= ozaki_max_exact_k, else OZ_ERR_ARG).  Adig [S][M][K], BTdig [S][N][K],
 * Q [G][M][N].  Uses context-owned scratch; synchronises the stream. */
int ozaki_pair_products(ozaki_ctx ctx, int64_t M, int64_t N, int64_t K, int slices, int ndiag,
                        const int8_t *Adig, const int8_t *BTdig, int32_t *Q, void *stream);

/* ---- two-site effective Hamiltonian -------------------------------- */
/* sigma = H_eff psi with H_eff = sum over triples of alpha L_op (x) R_op
 * restricted to symmetry blocks ("Theory of TNS/DMRG": the update of the
 * second subroutine diagonalises this operator on the two-site tensor).
 *
 * Layout: left sectors with sizes left_dim[n_left], right sectors with
 * right_dim[n_right], physical dimension phys (16 = d^2 for d = 4, or 1).
 * psi (and sigma, same layout) is a list of blocks; block b couples left
 * sector psi_lr[2b] with right sector psi_lr[2b+1] and is stored at element
 * offset psi_offset[b] as a [left_dim][phys][right_dim] row-major array.
 * L block i (operator L_key[3i], left sectors (L_key[3i+1], L_key[3i+2]))
 * is a left_dim x left_dim row-major matrix at L_offset[i] in L_data; R
 * blocks likewise with right sectors in R_data.  All arrays of the layout
 * struct are HOST arrays, copied by heff_plan_create.
 *
 * Triple t adds alpha * L[op][lo, li] psi[li, ri] R[op][ro, ri]^T to the
 * sigma block (lo, ro): per physical index j, a left GEMM
 * T = L[op][lo, li] Psi[li, ri] (Psi: the left_dim x phys*right_dim view),
 * then sigma' += alpha T' R^T (T', sigma': the left_dim*phys x right_dim
 * views).  Each sigma block starts at +0 and adds its triples in list order
 * as sigma = fma(alpha, c, sigma), so results do not depend on scheduling.
 * A non-null diag (device, laid out like psi) then adds sigma + diag * psi.
 * Dense two-site H_eff is one left and one right sector of size D, phys 16,
 * one psi block and triples (k, 0, 0, 0, 0, 1) for k < Kop. */
typedef struct {
    int32_t op, lo, li, ri, ro;
    double alpha;
} heff_triple;

typedef struct {
    int32_t n_left, n_right, phys;
    const int32_t *left_dim;    /* [n_left]  */
    const int32_t *right_dim;   /* [n_right] */
    int32_t n_psi_blocks;
    const int32_t *psi_lr;      /* [2 * n_psi_blocks] */
    const int64_t *psi_offset;  /* [n_psi_blocks] element offsets */
    int32_t n_L_blocks;
    const int32_t *L_key;       /* [3 * n_L_blocks] (op, lo, li) */
    const int64_t *L_offset;    /* [n_L_blocks] */
    int32_t n_R_blocks;
    const int32_t *R_key;       /* [3 * n_R_blocks] (op, ro, ri) */
    const int64_t *R_offset;    /* [n_R_blocks] */
} heff_layout;

/* Build a plan.  L_data / R_data / diag are device pointers that must stay
 * valid and unchanged for the plan's lifetime.  slices in [2, 8] caches the
 * int8 slices of every L and R block once (the operators are fixed during a
 * Davidson run); slices = 0 uses the native FP64 MFMA path.  triples is a
 * host array.  The plan owns every buffer it needs, so heff_apply never
 * allocates; the intermediates T take at most the context's heff budget
 * (ozaki_ctx_set_heff_budget) plus one first product.  Synchronises
 * `stream`. */
int heff_plan_create(ozaki_ctx ctx, heff_plan *out, const heff_layout *layout,
                     const double *L_data, const double *R_data, int32_t n_triples,
                     const heff_triple *triples, const double *diag, int slices, int ndiag,
                     void *stream);
/* sigma = H_eff psi (sigma overwritten; psi and sigma, n elements each,
 * must not overlap: OZ_ERR_ARG if their address ranges intersect).
 * One grouped launch per phase and chunk of the triple list; enqueue only.
 * Replay: the first apply with a given (psi, sigma) pair captures the
 * plan's launch sequence into a HIP graph (on a private stream; this creates
 * the graph, which takes host and driver resources) and later applies with
 * the same pair launch that graph on `stream`.  At most 96 graphs are kept
 * per plan; evicting the least recently used one synchronises `stream`.
 * The launches are issued directly instead when phase timing is on, when
 * `stream` is being captured by the caller, or after
 * heff_plan_set_graphs(plan, 0).  Results are identical either way.
 * Applies of one plan must not overlap in time (the plan's slice buffers
 * and tile counters are shared by its applies): issue them on one stream
 * or order the streams. */
int heff_apply(heff_plan plan, const double *psi, double *sigma, void *stream);
/* Enable (default) or disable graph replay in heff_apply. */
int heff_plan_set_graphs(heff_plan plan, int enable);
/* Number of graphs the plan currently holds. */
int heff_plan_graph_count(heff_plan plan);
/* Tile variants the plan's two grouped phases use (emulated plans; -1 for
 * native FP64 plans). */
int heff_plan_variants(heff_plan plan, int32_t *first, int32_t *second);
/* Launch kind of the plan's two grouped phases (0 one workgroup per tile,
 * 1 streamed, 2 resident, 3 paired terms; -1 for native FP64 plans). */
int heff_plan_launches(heff_plan plan, int32_t *first, int32_t *second);
/* Total elements of psi for the plan's layout. */
int64_t heff_vector_length(heff_plan plan);
/* The choice of grouped phase `phase` (0 = first product, 1 = second) in an
 * emulated plan: tile variant, order (0 XCD parts, 1 longest tile first,
 * 2 whole outputs per XCD) and
 * launch (0 one workgroup per tile, k > 0 streamed on k CUs,
 * OZ_HEFF_LAUNCH_RESIDENT resident, OZ_HEFF_LAUNCH_PAIRED_TERMS paired
 * terms); all -1 for a native FP64 plan. */
int heff_plan_phase(heff_plan plan, int phase, int32_t *variant, int32_t *order, int32_t *launch);
/* Number of chunks the plan's triple list runs in (ozaki_ctx_set_heff_budget). */
int heff_plan_chunks(heff_plan plan);
/* Device bytes the plan holds (all its allocations); *T_bytes (nullable)
 * gets the part that holds the intermediates T. */
int64_t heff_plan_bytes(heff_plan plan, int64_t *T_bytes);
/* FP64-equivalent flops of one heff_apply (2 m n k summed over all GEMMs). */
double heff_flops(heff_plan plan);
int heff_plan_destroy(heff_plan plan);

/* ---- Davidson eigensolver (lowest eigenpair) ------------------------ */
/* A standard Davidson iteration with diagonal preconditioner for the
 * Krylov diagonalisation of the second DMRG subroutine ("Theory of
 * TNS/DMRG"; convergence threshold on the residual as in "Numerical
 * procedure").  The matvec is heff_apply of H; orthogonalisation,
 * Rayleigh-Ritz and the residual run in FP64 on the device.
 * davidson_create: hdiag = diag(H) and x0 (device, heff_vector_length
 * elements) are copied; 2 <= m_max <= 64; allocates V and W (m_max vectors
 * each), normalises x0 and performs the first matvec.
 * davidson_step: one iteration (Rayleigh-Ritz on the current basis, Ritz
 * vector and residual, then, unless converged, preconditioned correction,
 * two classical Gram-Schmidt passes, one matvec).  Synchronises the stream
 * to fill *info (theta, residual norm, iteration, basis size, status) and
 * returns OZ_OK while running, or OZ_CONVERGED / OZ_STAGNATED / OZ_MAX_ITER.
 * The Rayleigh-Ritz solve of a step is issued at the end of the step before
 * (davidson_create issues the first), so a step reads (theta, rho) from a
 * pinned buffer, decides, and, when it continues, issues the correction,
 * the basis update, the matvec and the next Rayleigh-Ritz solve as one
 * replay of a graph captured per Ritz buffer (two in all: the basis size
 * lives on the device and the matvec runs on fixed buffers), then
 * synchronises once.  Replayed and directly issued steps give the same
 * bits.  Phase timing (ozaki_ctx_set_timing) issues the launches directly.
 * davidson_get_vector copies the Ritz vector of the theta the last step
 * reported (unit norm).
 * davidson_set_graphs: enable (default) or disable the graph replay;
 * davidson_graph_count: graphs the solver holds. */
typedef struct {
    double theta, resnorm;
    int32_t iter, m, status;
} davidson_info;

int davidson_create(ozaki_ctx ctx, davidson *out, heff_plan H, const double *hdiag,
                    const double *x0, int m_max, double tol, int max_iter, void *stream);
int davidson_step(davidson dav, davidson_info *info, void *stream);
int davidson_get_vector(davidson dav, double *x_out, void *stream);
int davidson_set_graphs(davidson dav, int enable);
int davidson_graph_count(davidson dav);
int davidson_destroy(davidson dav);

/* ---- Lanczos eigensolver (lowest eigenpair) ------------------------- */
/* The other Krylov method the paper runs for the same step ("Numerical
 * stability": Lanczos against Davidson at low slice counts and several
 * residual thresholds).  Lanczos with full reorthogonalisation (two
 * classical Gram-Schmidt passes against the whole basis) and explicit
 * restart: the tridiagonal T_m (alpha_j = q_j . H q_j from the first pass,
 * beta_j = |w_j|) is diagonalised on the host (cyclic Jacobi, m <= 64); the
 * residual estimate is beta_{m-1} |y_{m-1}| for the lowest Ritz pair
 * (theta, y).  When m reaches m_max the basis restarts from the Ritz vector.
 * The matvec is heff_apply of H; everything else is FP64 on the device.
 * lanczos_create: x0 (device, heff_vector_length elements) is copied and
 * normalised; 2 <= m_max <= 64; allocates m_max + 1 basis vectors.
 * lanczos_step: one matvec and one Ritz solve; synchronises the stream to
 * fill *info (theta, residual estimate, iteration, basis size, status);
 * returns OZ_OK while running, else OZ_CONVERGED (estimate <= tol or an
 * invariant subspace), OZ_STAGNATED (the last 20 estimates never below half
 * the best before them) or OZ_MAX_ITER.
 * lanczos_get_vector writes the current Ritz vector Q y (unit norm). */
typedef struct lanczos_s *lanczos;
int lanczos_create(ozaki_ctx ctx, lanczos *out, heff_plan H, const double *x0, int m_max, double tol,
                   int max_iter, void *stream);
int lanczos_step(lanczos lz, davidson_info *info, void *stream);
int lanczos_get_vector(lanczos lz, double *x_out, void *stream);
int lanczos_destroy(lanczos lz);

/* ---- DMRG truncation and renormalisation --------------------------- */
/* The two steps beside the H_eff diagonalisation in a site update: the
 * eigenvalue decomposition of the reduced density matrix rho = Psi Psi^T
 * (its dominant eigenvectors form the kept basis U, "Algorithm" and the
 * numerical-stability discussion of the paper) and the renormalisation of
 * block operators into that basis (network contraction by GEMMs).  The
 * paper runs both with native and with emulated FP64; both take (slices,
 * ndiag) like ozaki_dgemm, slices = 0 meaning native FP64.
 *
 * rdm_eig: eigenpairs of a symmetric n x n matrix (a reduced density
 * matrix) by two-sided block Jacobi on the device (n <= 8192; blocks of 32
 * rows, padded to n_p = roundup(n, 64)).  A sweep runs n_p/32 - 1 rounds;
 * a round diagonalises the 64 x 64 diagonal blocks of the paired blocks of
 * M = W A W^T (cyclic Jacobi, one workgroup per pair, in FP64) and applies
 * the rotations to the rows and columns of M and to the basis W: three
 * grouped GEMMs of inner length 64 in the plan's arithmetic (emulated with
 * (slices, ndiag), or native FP64 for slices = 0).
 * rdm_eig_create allocates 4 n_p^2 doubles plus, when emulated, 2 S n_p^2
 * bytes of slices.  OZ_ERR_ARG for n outside 1..8192 or bad (slices, ndiag).
 * rdm_eig_solve: A (device, row-major, lda >= n) is read, not modified;
 * writes the nev largest eigenvalues in decreasing order to evals (device,
 * nev doubles) and their unit eigenvectors as the columns of Z (device,
 * n x nev row-major, ldz >= nev).  tol = 0 selects 4 sqrt(n_p) u, with u
 * the unit roundoff of the arithmetic (2^-53, or 2^(1-8S) when emulated).
 * The iteration ends when a whole sweep meets no off-diagonal entry of M
 * larger than tol |A|_F (absolute accuracy, as a tridiagonal-based solver
 * gives), when three sweeps in a row fail to halve the best off-diagonal
 * mass (the arithmetic's floor), or after max_sweeps.  With nev < n the
 * couplings between two rows outside the wanted part (diagonal below the
 * middle of the gap at the nev-th value of the previous sweep) are exempt
 * from tol, provided their Frobenius mass cannot lift an unwanted eigenvalue
 * above the nev-th one (Weyl's bound): the tail of a graded spectrum is not
 * resolved beyond what the kept eigenpairs need.  info (may be NULL):
 * sweeps run, status (OZ_CONVERGED, OZ_STAGNATED or OZ_MAX_ITER), the last
 * sweep's largest off-diagonal entry over |A|_F and the sum of all n
 * eigenvalues.  Results are written in all three cases.  The upper triangle
 * of the diagonal blocks is used where symmetry is assumed; NaN or Inf in
 * A: OZ_ERR_ARG.  Synchronises the stream.  One solve at a time per plan. */
typedef struct rdm_eig_s *rdm_eig;
typedef struct {
    int32_t sweeps, status;
    double off;    /* largest off-diagonal entry of the last sweep over |A|_F */
    double trace;  /* sum of all n eigenvalues (discarded weight = trace - kept sum) */
} rdm_eig_info;
int rdm_eig_create(ozaki_ctx ctx, rdm_eig *out, int64_t n, int slices, int ndiag);
int rdm_eig_solve(rdm_eig plan, const double *A, int64_t lda, int64_t nev, double *evals, double *Z,
                  int64_t ldz, double tol, int max_sweeps, rdm_eig_info *info, void *stream);
int rdm_eig_destroy(rdm_eig plan);

/* ozaki_renormalize: O'_k = U^T O_k U for k < count, with U (device, n x D
 * row-major, ldu >= D, D <= n), O_k (device pointers in the host array ops,
 * n x n, ldo >= n) and O'_k (device pointers in outs, D x D, ldout >= D).
 * Two GEMMs per operator, T = O_k U then U^T T, each an ozaki_dgemm with
 * the given (slices, ndiag) (slices = 0: native FP64), so the results are
 * those of the two ozaki_dgemm calls.  workspace: device, 256-byte aligned,
 * ozaki_renormalize_workspace_bytes(n, D, slices, ndiag) bytes (the
 * intermediate T and the GEMM workspace).  Asynchronous on the stream. */
size_t ozaki_renormalize_workspace_bytes(int64_t n, int64_t D, int slices, int ndiag);
int ozaki_renormalize(ozaki_ctx ctx, int64_t n, int64_t D, const double *U, int64_t ldu, int count,
                      const double *const *ops, int64_t ldo, double *const *outs, int64_t ldout, int slices,
                      int ndiag, void *workspace, size_t workspace_bytes, void *stream);

#ifdef __cplusplus
}
#endif
#endif /* OZAKI_H */
