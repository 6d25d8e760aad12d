// Internal declarations shared by the HIP kernels and the host runtime.
//
// Packed slice layout (the operand format of the int8 pair GEMM).  An
// operand with R rows (rows of op(A), or columns of op(B)) and inner length
// K is stored as S int8 digit planes, padded to Rp = roundup(R, 32) rows and
// Kp = roundup(K, 32).  Byte (r, k) of slice s lives at
//
//     ((k / 32 * S + s) * 2 + (k / 16) % 2) * Rp * 16 + r * 16 + k % 16
//
// i.e. for every 32-wide K block and slice there are two runs of Rp 16-byte
// chunks.  A run of consecutive rows is contiguous, so a tile load is a
// straight copy of 2S runs, and the LDS image of a tile (same order) gives
// each 32x32x32 int8 MFMA operand as 1 KiB read by consecutive lanes.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace oz {

constexpr int kKB = 32;      // inner-dimension block of the packed layout
constexpr int kRowQ = 32;    // row granularity of the packed layout
// The pair kernels address one packed K block of an operand (2S runs of
// rows_p 16-byte chunks) with 32-bit buffer offsets: rows_p is bounded so
// that 2 * 8 * rows_p * 16 stays below 2^31.
constexpr int64_t kMaxPackedRows = (INT32_MAX / (2 * 8 * 16)) / kRowQ * kRowQ;
constexpr int32_t kExpBad = INT32_MIN;
// Codes of the fused row-exponent maxima (an exponent code is the shared
// exponent of one element's magnitude): an all-zero group, a NaN or +-Inf.
constexpr int32_t kEmaxZero = INT32_MIN + 1;
constexpr int32_t kEmaxNaN = INT32_MAX;

// Exponent e of a group whose largest magnitude is mu: with mu = m 2^E,
// m in [0.5, 1), e = E + [m > 127/128], so |x| 2^(8S-1-e) <= 127 256^(S-1)
// and the leading slice fits in int8.  Computed from the bit pattern.  It is
// non-decreasing in mu, so the largest exponent of a group's elements is the
// exponent of its largest magnitude.
__device__ inline int32_t shared_exponent(double mu) {
    if (mu == 0.0) return 0;
    const uint64_t b = static_cast<uint64_t>(__double_as_longlong(mu));
    const int be = static_cast<int>((b >> 52) & 0x7ff);
    const uint64_t fr = b & ((1ull << 52) - 1);
    if (be != 0) return be - 1022 + (fr > (63ull << 46) ? 1 : 0);
    // subnormal: mu = fr 2^-1074 with top bit p; frexp gives E = p - 1073, m = fr / 2^(p+1)
    const int p = 63 - __clzll(static_cast<long long>(fr));
    return p - 1073 + ((fr << 7) > (127ull << (p + 1)) ? 1 : 0);
}

inline int64_t round_up(int64_t x, int64_t m) { return (x + m - 1) / m * m; }
inline int64_t ceil_div(int64_t x, int64_t m) { return (x + m - 1) / m; }

// One product contributing to an output tile: c = ozaki(A rows, B rows), weight alpha.
struct TermDesc {
    const int8_t *A;       // packed A operand (rows = rows of op(A))
    const int32_t *e;      // its row exponents
    const int8_t *B;       // packed B operand (rows = columns of op(B))
    const int32_t *f;      // its column exponents
    int64_t a_rows_p;      // padded row count of A's packed planes
    int64_t b_rows_p;      // padded row count of B's packed planes
    int32_t kblocks;       // Kp / 32
    int32_t pad_;
    double alpha;
};

// A BM x BN output tile and the list of terms summed into it.
struct TileDesc {
    int32_t term_begin, term_end;
    int32_t m0, n0;        // tile origin (also the row offsets into A and B)
    int32_t out;           // index of the output matrix
    int32_t pad_;
};

struct OutDesc {
    double *C;
    int64_t ldc;
    int32_t M, N;          // valid extent (stores outside are skipped)
    // GEMM mode, nullable: exponent-code maxima of the stored values, element
    // (i, j) into emax[i * ep + j / en] (en a multiple of 32, or ep = 1 and
    // en >= N), combined with atomic max
    int32_t *emax;
    int32_t ep, en;
    // accumulating mode: 1 = the running sum starts from the stored C (a term
    // list split over launches continues where the previous launch stopped),
    // 0 = it starts from +0
    int32_t cont;
    int32_t pad_;
};

enum PairMode : int32_t {
    kModeGemm = 0,     // one term; C = alpha*c (beta == 0) or fma(alpha, c, beta*C)
    kModeAccum = 1,    // term list; sigma = +0, then sigma = fma(alpha_t, c_t, sigma)
    kModeQ = 2,        // one term; write the int32 diagonal sums Q[g][i][j]
    kModeQ64 = 3,      // one term over one K chunk; store (qw_first) or add its sums to Qw
};

// Counters of one streamed launch: a tile counter per XCD, then the number
// of workgroups that found their queue empty.
constexpr int kStreamQueueInts = 16;

struct PairArgs {
    // grouped launch
    const TileDesc *tiles;
    const TermDesc *terms;
    const OutDesc *outs;
    int32_t ntiles;
    // single-GEMM launch (tiles from the grid)
    int32_t tiles_n;
    TermDesc term;
    OutDesc out;
    int32_t mode;
    int32_t qw_first;      // kModeQ64: first chunk stores instead of adding
    double beta;
    int32_t *Q;            // kModeQ output, [G][M][N]
    double *out_base;      // grouped: when set, OutDesc::C holds an element offset from it
    // int64 partial sums [G][tiles_m*BM][tiles_n*BN] of earlier K chunks when
    // K exceeds the exact int32 range; added in the kModeGemm epilogue if set
    int64_t *Qw;
    int64_t qw_ld;         // leading dimension of one Qw plane (tiles_n * BN)
    int64_t qw_plane;      // elements per Qw plane
    // grouped: 0 = one workgroup per listed tile; > 0 = the streamed kernel,
    // resident workgroups on this many compute units taking tiles from
    // `queue` (kStreamQueueInts zeroed ints, left zeroed by every launch)
    int32_t stream_cus;
    int32_t *queue;
    // grouped, GEMM mode with beta = 0: nwg > 0 = the resident kernel, nwg
    // workgroups (all resident at once), workgroup b taking the tiles
    // tiles[wg_off[b] .. wg_off[b + 1]) in order
    int32_t nwg;
    const int32_t *wg_off;
    // grouped, accumulating mode on the 64 x 64 tiles of variant 0: 1 = the
    // paired-term kernel (eight waves per tile, two terms at a time)
    int32_t terms2;
};

// FP64 GEMM term: op(A) (M x K) times op(B) (K x N), both plain FP64.
struct Term64 {
    const double *A;
    const double *B;
    int64_t lda, ldb;
    int32_t K;
    int32_t pad_;
    double alpha;
};

struct Dgemm64Args {
    const TileDesc *tiles;
    const Term64 *terms;
    const OutDesc *outs;
    int32_t ntiles;
    int32_t tiles_n;
    Term64 term;
    OutDesc out;
    int32_t mode;          // kModeGemm or kModeAccum
    int32_t tile;          // grouped: edge of the listed tiles (64 or 128, see dgemm_tile_for)
    double beta;
    double *out_base;      // grouped: when set, OutDesc::C holds an element offset from it
    const double *b_base;  // grouped: when set, Term64::B holds an element offset from it
};

// Grouped slicing: many blocks in one launch.  Offsets are relative to base
// pointers passed at launch, so the same descriptors serve every call.
struct SliceBlock {
    int64_t x_off;   // element offset of the block from the FP64 base
    int64_t ld;      // leading dimension of the stored block
    int32_t R, K;    // groups (rows of the packed operand) and inner length
    int32_t trans;   // 0: stored R x K (groups are rows); 1: stored K x R (groups are columns)
    int32_t pad_;
    int64_t e_off;   // int32 offset of the group exponents from the exponent base
    int64_t p_off;   // byte offset of the packed planes from the packed base
    int64_t Rp;      // padded group count of the packed planes
};
// Work per task of the grouped exponent and slice launches: 16 rows or 64
// columns per exponent task, 32 groups x 8 K blocks per slice task.
constexpr int kExpTaskRows = 16;
constexpr int kExpTaskCols = 64;
constexpr int kSliceTaskKB = 8;
// Column exponent tasks of sets built with split columns cover this many
// rows each and combine their maxima through exponent codes (atomic max).
constexpr int kExpColChunk = 128;

struct SliceTask {
    int32_t block;
    int32_t a;       // exponent task: first group; slice task: first group (32-aligned)
    int32_t b;       // slice task: 32-wide K block index; split column task: row chunk
    int32_t pad_;
};

// ---- launchers ---------------------------------------------------------
// Shared exponents of each row of X (R x K, row-major, ld): e[r], flag on NaN/Inf.
hipError_t launch_row_exponents(const double *X, int64_t ld, int64_t R, int64_t K, int32_t *e,
                                uint32_t *flag, hipStream_t s);
// Shared exponents of each column of X (K x R, row-major, ld).  part: scratch
// of col_exponent_scratch(K, R) bytes.
size_t col_exponent_scratch(int64_t K, int64_t R);
hipError_t launch_col_exponents(const double *X, int64_t ld, int64_t K, int64_t R, int32_t *e,
                                double *part, uint32_t *flag, hipStream_t s);
// Sum of squares of each group: rows of X (R x K) when by_rows, else columns
// of X (K x R, part: col_exponent_scratch(K, R) bytes).
hipError_t launch_group_sumsq(bool by_rows, const double *X, int64_t ld, int64_t R, int64_t K, double *ss,
                              double *part, hipStream_t s);
// Slice X into the packed layout.  trans = false: X is R x K (groups are rows);
// trans = true: X is K x R (groups are columns).  Pads rows to Rp, K to Kp with 0.
hipError_t launch_slice(int S, bool trans, const double *X, int64_t ld, int64_t R, int64_t K,
                        const int32_t *e, int8_t *packed, int64_t Rp, hipStream_t s);
// Grouped exponent pass (tasks of kExpTaskRows rows or kExpTaskCols columns)
// and slice pass (tasks of 32 groups x kSliceTaskKB 32-wide K blocks).
// With emax_base (column tasks split into row chunks of kExpColChunk), the
// column tasks combine exponent codes into emax_base[e_off + group] with
// atomic max instead of writing exponents; launch_emax_finish completes them.
hipError_t launch_exponents_grouped(const SliceBlock *blocks, const SliceTask *tasks, int ntasks,
                                    const double *x_base, int32_t *e_base, uint32_t *flag,
                                    hipStream_t s, int32_t *emax_base = nullptr);
// Exponents from code maxima left in emax by a GEMM-mode pair launch
// (OutDesc::emax) or a split column exponent pass; emax is left at kEmaxZero.
hipError_t launch_emax_finish(int32_t *emax, int32_t *e, int64_t n, uint32_t *flag, hipStream_t s);
hipError_t launch_slice_grouped(int S, const SliceBlock *blocks, const SliceTask *tasks, int ntasks,
                                const double *x_base, const int32_t *e_base, int8_t *p_base,
                                hipStream_t s);
// Debug conversions between [S][R][K] digits and the packed layout.
hipError_t launch_pack(int S, const int8_t *canon, int64_t R, int64_t K, int8_t *packed,
                       int64_t Rp, hipStream_t s);
hipError_t launch_unpack(int S, const int8_t *packed, int64_t Rp, int64_t R, int64_t K,
                         int8_t *canon, hipStream_t s);

// Tile variants of the int8 pair GEMM.  v < 0 selects the default variant.
struct PairShape { int bm, bn; };
bool pair_supported(int S, int G);
int pair_num_variants();
bool pair_variant_ok(int G, int v);
int pair_default_variant(int G);
PairShape pair_shape(int S, int G, int v);
hipError_t launch_pair_single(int S, int G, int v, const PairArgs &a, int tiles_m, hipStream_t s);
hipError_t launch_pair_grouped(int S, int G, int v, const PairArgs &a, hipStream_t s);
// Workgroups of the resident GEMM-mode kernel that fit on one compute unit
// at once for (S, G, v); 0 where that kernel is not built for the variant.
int pair_resident_per_cu(int S, int G, int v);
// Whether the paired-term accumulating kernel is built for (S, G, v).
bool pair_terms2_ok(int S, int G, int v);

// FP64 MFMA GEMM.  The single launch picks its tile size from the output
// extent (a.out) and the compute-unit count; the grouped launch takes tiles
// of edge a.tile (64 or 128), one workgroup per listed tile.
// dgemm_tile_for: the edge for a set of outputs with `tiles128` tiles of 128.
int dgemm_tile_for(int64_t tiles128, int num_cu);
hipError_t launch_dgemm_single(bool ta, bool tb, const Dgemm64Args &a, int num_cu, hipStream_t s);
hipError_t launch_dgemm_grouped(bool tb, const Dgemm64Args &a, hipStream_t s);

// sigma[i] = sigma[i] + diag[i] * psi[i] (two roundings), i < n.
hipError_t launch_diag_axpy(const double *diag, const double *psi, double *sigma, int64_t n,
                            hipStream_t s);

}  // namespace oz
