// Two-site effective-Hamiltonian application sigma = H_eff psi
// ("Theory of TNS/DMRG": the second subroutine's Krylov solver applies this
// operator to the two-site tensor of shape (D, d = 4, 4, D)).
//
// H_eff is a list of triples (op, lo, li, ri, ro, alpha); triple t adds
// alpha L[op][lo, li] psi[li, ri] R[op][ro, ri]^T to sigma block (lo, ro).  A
// dense two-site problem is one left and one right sector with phys = 16.
//
// Plan (built once per operator set):
//  * distinct left products u = (op, lo, li, ri): T_u = L[op][lo, li] Psi[li, ri]
//    with Psi the left x (phys * right) view of a psi block;
//  * every sigma block is split into tiles; a tile owns its output and sums
//    its triples' second products T'_u R^T (T'_u: the (left * phys) x right
//    view of T_u) in list order, sigma = fma(alpha, c, sigma) from +0, so the
//    result does not depend on scheduling and needs no atomics;
//  * emulated mode: the int8 slices of every L and R block are made once here;
//    psi and T are sliced on every apply (psi by columns, T by rows);
//  * the intermediates T_u live in a buffer of bounded size: the triple list
//    is cut into contiguous chunks whose distinct first products fit it
//    (ozaki_ctx_set_heff_budget), and the chunks run one after the other;
//    a sigma tile that already summed triples in an earlier chunk continues
//    from its stored value, so the sum is the same fma chain in list order.
// Apply = psi's exponents and slices, then per chunk: grouped first product,
// exponents + slices of its T, grouped second product; then the diagonal
// term.  Nothing is allocated or synchronised, so it can be captured.
#include <algorithm>
#include <map>
#include <tuple>
#include <vector>

#include "runtime.h"

using namespace oz;

// One chunk of the triple list: its first products write into the shared T
// buffer, whose slices and exponents are shared too (chunks run in order).
struct HeffChunk {
    // emulated path
    SliceBlock *T_blocks = nullptr;
    SliceTask *T_etasks = nullptr, *T_stasks = nullptr;
    int n_T_etasks = 0, n_T_stasks = 0;
    bool fuse_T = false;      // T's exponents from the first phase's maxima
    int64_t T_e_total = 0;
    PairArgs argsL{}, argsR{};
    // FP64 path
    Dgemm64Args d64L{}, d64R{};
};

struct heff_plan_s {
    ozaki_ctx ctx = nullptr;
    int S = 0, G = 0;  // S == 0: native FP64 path
    int64_t n = 0;     // elements of psi / sigma
    double flops = 0;
    const double *diag = nullptr;
    std::vector<void *> allocs;
    // emulated path
    SliceBlock *psi_blocks = nullptr;
    SliceTask *psi_etasks = nullptr, *psi_stasks = nullptr;
    int n_psi_etasks = 0, n_psi_stasks = 0;
    int32_t *psi_e = nullptr;
    int8_t *psi_p = nullptr;
    double *T = nullptr;         // shared by the chunks
    int32_t *T_e = nullptr;
    int8_t *T_p = nullptr;
    int32_t *T_emax = nullptr;   // exponent-code maxima left by the first phase
    int32_t *psi_emax = nullptr;  // exponent-code maxima of psi's split column pass
    int64_t psi_e_total = 0;
    int varL = -1, varR = -1;   // tile variants of the two grouped phases
    int choice[2][3] = {{-1, -1, -1}, {-1, -1, -1}};  // per phase: variant, order, launch
    std::vector<HeffChunk> chunks;
    size_t T_bytes = 0;         // T buffer, its slices and exponents
    size_t bytes = 0;           // every device allocation of the plan
    // Replay: one instantiated graph of the apply sequence per (psi, sigma)
    // pair, captured on a private stream the first time the pair is seen.
    struct GraphSlot {
        const double *psi;
        double *sigma;
        hipGraphExec_t exec;
        uint64_t used;
    };
    bool use_graphs = true;
    hipStream_t cap = nullptr;
    std::vector<GraphSlot> graphs;
    uint64_t clock = 0;
};

namespace {

template <typename T>
int upload(heff_plan p, const std::vector<T> &v, T **out) {
    *out = nullptr;
    if (v.empty()) return OZ_OK;
    void *d = nullptr;
    hipError_t e = hipMalloc(&d, sizeof(T) * v.size());
    if (e != hipSuccess) return fail(OZ_ERR_NOMEM, "heff_plan_create: %zu bytes: %s", sizeof(T) * v.size(), hipGetErrorString(e));
    p->allocs.push_back(d);
    p->bytes += sizeof(T) * v.size();
    if ((e = hipMemcpy(d, v.data(), sizeof(T) * v.size(), hipMemcpyHostToDevice)) != hipSuccess)
        return hip_fail(e, "heff_plan_create: upload");
    *out = static_cast<T *>(d);
    return OZ_OK;
}

int alloc(heff_plan p, size_t bytes, void **out) {
    *out = nullptr;
    if (bytes == 0) return OZ_OK;
    hipError_t e = hipMalloc(out, bytes);
    if (e != hipSuccess) return fail(OZ_ERR_NOMEM, "heff_plan_create: %zu bytes: %s", bytes, hipGetErrorString(e));
    p->allocs.push_back(*out);
    p->bytes += bytes;
    return OZ_OK;
}

void free_plan(heff_plan p) {
    for (auto &g : p->graphs) hipGraphExecDestroy(g.exec);
    if (p->cap) hipStreamDestroy(p->cap);
    for (void *d : p->allocs) hipFree(d);
    delete p;
}

// Slice a set of blocks of x_base once (plan creation): grouped exponent and
// slice launches into freshly allocated exponent / packed buffers.
int slice_once(heff_plan p, const SliceSet &set, const double *x_base, int S, hipStream_t s,
               int32_t **e_out, int8_t **p_out) {
    int rc;
    SliceBlock *db;
    SliceTask *de, *ds;
    void *e_mem, *p_mem;
    if ((rc = upload(p, set.blocks, &db)) || (rc = upload(p, set.etasks, &de)) ||
        (rc = upload(p, set.stasks, &ds)))
        return rc;
    if ((rc = alloc(p, sizeof(int32_t) * std::max<int64_t>(set.e_total, 1), &e_mem)) ||
        (rc = alloc(p, std::max<int64_t>(set.p_total, 256), &p_mem)))
        return rc;
    hipError_t e;
    if ((e = launch_exponents_grouped(db, de, static_cast<int>(set.etasks.size()), x_base,
                                      static_cast<int32_t *>(e_mem), p->ctx->d_flags, s)) != hipSuccess)
        return hip_fail(e, "heff_plan_create: exponents");
    if ((e = launch_slice_grouped(S, db, ds, static_cast<int>(set.stasks.size()), x_base,
                                  static_cast<int32_t *>(e_mem), static_cast<int8_t *>(p_mem), s)) != hipSuccess)
        return hip_fail(e, "heff_plan_create: slices");
    *e_out = static_cast<int32_t *>(e_mem);
    *p_out = static_cast<int8_t *>(p_mem);
    return OZ_OK;
}

struct TileWork {
    TileDesc td;
    int64_t cost;
};

// The tiles of one output of M x N in a walk that keeps the blocks running
// together on one XCD close in both operands: groups of tile rows (fewer for
// tall tiles), column by column inside a group.
template <typename Make>
void walk_output(int64_t M, int64_t N, const PairShape &sh, Make make, std::vector<TileWork> *w) {
    const int64_t tm_n = ceil_div(M, sh.bm), tn_n = ceil_div(N, sh.bn);
    const int64_t group = sh.bm >= 2 * sh.bn ? 4 : 8;
    for (int64_t first = 0; first < tm_n; first += group) {
        const int64_t rows = std::min(group, tm_n - first);
        for (int64_t q = 0; q < rows * tn_n; ++q)
            w->push_back(make((first + q % rows) * sh.bm, (q / rows) * sh.bn));
    }
}

constexpr int kXcds = 8;

// Workgroup b of a launch runs on XCD b % 8.  Outputs are taken longest
// tile first (each output's tiles stay together in their walk), the list is
// cut into 8 contiguous parts of about equal cost and interleaved, so every
// XCD walks its own part in order; shorter parts are padded with empty tiles
// (output -1), which exit at once.
// Longest tile first over all outputs: for tiles of very different cost the
// hardware's own balancing over the XCDs does better than fixed parts.
void longest_first(const std::vector<std::vector<TileWork>> &outputs, std::vector<TileDesc> *out,
                   std::vector<int64_t> *cost) {
    std::vector<TileWork> all;
    for (auto &o : outputs) all.insert(all.end(), o.begin(), o.end());
    std::stable_sort(all.begin(), all.end(), [](const TileWork &a, const TileWork &b) { return a.cost > b.cost; });
    out->clear();
    cost->clear();
    for (auto &t : all) {
        out->push_back(t.td);
        cost->push_back(t.cost);
    }
}

void xcd_order(std::vector<std::vector<TileWork>> &outputs, std::vector<TileDesc> *out,
               std::vector<int64_t> *cost) {
    std::stable_sort(outputs.begin(), outputs.end(), [](const std::vector<TileWork> &a, const std::vector<TileWork> &b) {
        const int64_t ca = a.empty() ? 0 : a.front().cost, cb = b.empty() ? 0 : b.front().cost;
        return ca > cb;
    });
    std::vector<TileWork> all;
    int64_t total = 0;
    for (auto &o : outputs)
        for (auto &t : o) {
            all.push_back(t);
            total += t.cost;
        }
    std::vector<std::vector<TileWork>> part(kXcds);
    int64_t run = 0;
    size_t x = 0;
    for (auto &t : all) {
        // the part whose share of the cost this tile starts in
        while (x + 1 < part.size() && run * kXcds >= total * static_cast<int64_t>(x + 1)) ++x;
        part[x].push_back(t);
        run += t.cost;
    }
    size_t longest = 0;
    for (auto &p : part) longest = std::max(longest, p.size());
    out->clear();
    cost->clear();
    for (size_t i = 0; i < longest; ++i)
        for (auto &p : part) {
            if (i < p.size()) {
                out->push_back(p[i].td);
                cost->push_back(p[i].cost);
            } else {
                out->push_back(TileDesc{0, 0, 0, 0, -1, 0});
                cost->push_back(0);
            }
        }
}

// Whole outputs to XCDs, heaviest first, each to the XCD with the least
// cost so far (longest processing time first); every XCD walks the tiles of
// its outputs in that order.  The tiles of one output then run side by side
// on one XCD and share its L2 (their row and column panels), while the XCDs
// stay balanced to within one output.
void output_lpt_order(const std::vector<std::vector<TileWork>> &outputs, std::vector<TileDesc> *out,
                      std::vector<int64_t> *cost) {
    std::vector<int64_t> oc(outputs.size(), 0);
    std::vector<size_t> idx;
    for (size_t i = 0; i < outputs.size(); ++i) {
        for (auto &t : outputs[i]) oc[i] += t.cost;
        if (!outputs[i].empty()) idx.push_back(i);
    }
    std::stable_sort(idx.begin(), idx.end(), [&](size_t a, size_t b) { return oc[a] > oc[b]; });
    std::vector<std::vector<TileWork>> part(kXcds);
    std::vector<int64_t> load(kXcds, 0);
    for (size_t i : idx) {
        const size_t x = static_cast<size_t>(std::min_element(load.begin(), load.end()) - load.begin());
        part[x].insert(part[x].end(), outputs[i].begin(), outputs[i].end());
        load[x] += oc[i];
    }
    size_t longest = 0;
    for (auto &p : part) longest = std::max(longest, p.size());
    out->clear();
    cost->clear();
    for (size_t i = 0; i < longest; ++i)
        for (auto &p : part) {
            if (i < p.size()) {
                out->push_back(p[i].td);
                cost->push_back(p[i].cost);
            } else {
                out->push_back(TileDesc{0, 0, 0, 0, -1, 0});
                cost->push_back(0);
            }
        }
}

constexpr int kHeffLaunchResident = OZ_HEFF_LAUNCH_RESIDENT;
constexpr int kHeffLaunchPairedTerms = OZ_HEFF_LAUNCH_PAIRED_TERMS;
// workgroups per compute unit the resident schedules are built for, at most
constexpr int kMaxResidentPerCu = 8;

// The fixed cost of starting a tile in a resident schedule, in the tile
// costs' unit (K blocks times the tile's area): about two K blocks.
int64_t resident_start_cost(const PairShape &sh) { return 2 * static_cast<int64_t>(sh.bm) * sh.bn; }

// Schedule of the resident kernel over a tile list: nwg workgroups, all on
// the device at once, workgroup b on XCD b % 8.  Each listed tile goes to
// the XCD its list position names (position p to XCD p % 8, as in the
// launch with one workgroup per tile), there to the workgroup with the least
// cost so far, in list order.  *out gets the tiles of workgroup 0, 1, ... in
// order, *off the nwg + 1 offsets of their runs.
void resident_schedule(const std::vector<TileDesc> &tl, const std::vector<int64_t> &cost, int nwg,
                       int64_t start_cost, std::vector<TileDesc> *out, std::vector<int32_t> *off) {
    std::vector<std::vector<TileDesc>> per(static_cast<size_t>(nwg));
    std::vector<int64_t> load(static_cast<size_t>(nwg), 0);
    for (size_t p = 0; p < tl.size(); ++p) {
        if (tl[p].out < 0) continue;
        int best = -1;
        for (int b = static_cast<int>(p % kXcds); b < nwg; b += kXcds)
            if (best < 0 || load[b] < load[best]) best = b;
        if (best < 0) best = static_cast<int>(p % static_cast<size_t>(nwg));
        per[best].push_back(tl[p]);
        load[best] += cost[p] + start_cost;
    }
    out->clear();
    off->assign(1, 0);
    for (auto &v : per) {
        out->insert(out->end(), v.begin(), v.end());
        off->push_back(static_cast<int32_t>(out->size()));
    }
}

}  // namespace

extern "C" {

int heff_plan_create(ozaki_ctx ctx, heff_plan *out, const heff_layout *L, const double *L_data,
                     const double *R_data, int32_t n_triples, const heff_triple *triples,
                     const double *diag, int slices, int ndiag, void *stream) {
    if (!out) return fail(OZ_ERR_ARG, "heff_plan_create: out is NULL");
    *out = nullptr;
    if (!ctx || !L) return fail(OZ_ERR_ARG, "heff_plan_create: NULL ctx or layout");
    if (slices != 0 && (slices < 2 || slices > 8)) return fail(OZ_ERR_ARG, "heff_plan_create: slices = %d", slices);
    const int S = slices;
    const int G = S ? resolve_ndiag(S, ndiag) : 0;
    if (S && !valid_sg(S, G)) return fail(OZ_ERR_ARG, "heff_plan_create: ndiag = %d", ndiag);
    if (L->n_left < 1 || L->n_right < 1 || L->phys < 1 || !L->left_dim || !L->right_dim)
        return fail(OZ_ERR_ARG, "heff_plan_create: empty sector list");
    if (n_triples < 0 || (n_triples > 0 && !triples)) return fail(OZ_ERR_ARG, "heff_plan_create: triples");
    const int64_t p = L->phys;
    std::vector<int64_t> ld(L->left_dim, L->left_dim + L->n_left), rd(L->right_dim, L->right_dim + L->n_right);
    for (auto d : ld) if (d < 1) return fail(OZ_ERR_ARG, "heff_plan_create: left sector size %lld", (long long)d);
    for (auto d : rd) if (d < 1) return fail(OZ_ERR_ARG, "heff_plan_create: right sector size %lld", (long long)d);
    // every operand of the two products has at most phys * (largest sector) rows
    {
        int64_t big = 1;
        for (auto d : ld) big = std::max(big, d);
        for (auto d : rd) big = std::max(big, d);
        if (round_up(big * std::max<int64_t>(L->phys, 1), kRowQ) > kMaxPackedRows)
            return fail(OZ_ERR_ARG, "heff_plan_create: phys * sector size above %lld", (long long)kMaxPackedRows);
    }

    // psi / sigma blocks
    std::map<std::pair<int, int>, int> psi_of;
    std::vector<std::pair<int64_t, int64_t>> extents;
    int64_t n = 0;
    for (int b = 0; b < L->n_psi_blocks; ++b) {
        const int l = L->psi_lr[2 * b], r = L->psi_lr[2 * b + 1];
        if (l < 0 || l >= L->n_left || r < 0 || r >= L->n_right) return fail(OZ_ERR_ARG, "heff_plan_create: psi block %d sectors", b);
        if (psi_of.count({l, r})) return fail(OZ_ERR_ARG, "heff_plan_create: psi block (%d, %d) repeated", l, r);
        if (L->psi_offset[b] < 0) return fail(OZ_ERR_ARG, "heff_plan_create: psi offset");
        psi_of[{l, r}] = b;
        const int64_t sz = ld[l] * p * rd[r];
        extents.push_back({L->psi_offset[b], L->psi_offset[b] + sz});
        n = std::max(n, L->psi_offset[b] + sz);
    }
    std::sort(extents.begin(), extents.end());
    for (size_t i = 1; i < extents.size(); ++i)
        if (extents[i].first < extents[i - 1].second) return fail(OZ_ERR_ARG, "heff_plan_create: psi blocks overlap");
    std::map<std::tuple<int, int, int>, int> L_of, R_of;
    for (int i = 0; i < L->n_L_blocks; ++i) {
        auto key = std::make_tuple(L->L_key[3 * i], L->L_key[3 * i + 1], L->L_key[3 * i + 2]);
        if (std::get<1>(key) < 0 || std::get<1>(key) >= L->n_left || std::get<2>(key) < 0 || std::get<2>(key) >= L->n_left)
            return fail(OZ_ERR_ARG, "heff_plan_create: L block %d sectors", i);
        L_of[key] = i;
    }
    for (int i = 0; i < L->n_R_blocks; ++i) {
        auto key = std::make_tuple(L->R_key[3 * i], L->R_key[3 * i + 1], L->R_key[3 * i + 2]);
        if (std::get<1>(key) < 0 || std::get<1>(key) >= L->n_right || std::get<2>(key) < 0 || std::get<2>(key) >= L->n_right)
            return fail(OZ_ERR_ARG, "heff_plan_create: R block %d sectors", i);
        R_of[key] = i;
    }
    if ((L->n_L_blocks > 0 && !L_data) || (L->n_R_blocks > 0 && !R_data)) return fail(OZ_ERR_ARG, "heff_plan_create: L_data / R_data NULL");

    // distinct left products and the triple list's sigma blocks
    std::map<std::tuple<int, int, int, int>, int> u_of;
    struct U { int op, lo, li, ri, Lb, psib; };
    std::vector<U> us;
    std::vector<int> tri_u(n_triples), tri_R(n_triples), tri_sigma(n_triples);
    double flops = 0;
    for (int t = 0; t < n_triples; ++t) {
        const heff_triple &tr = triples[t];
        auto lk = std::make_tuple(tr.op, tr.lo, tr.li);
        auto rk = std::make_tuple(tr.op, tr.ro, tr.ri);
        if (!L_of.count(lk)) return fail(OZ_ERR_ARG, "heff_plan_create: triple %d: no L block (%d, %d, %d)", t, tr.op, tr.lo, tr.li);
        if (!R_of.count(rk)) return fail(OZ_ERR_ARG, "heff_plan_create: triple %d: no R block (%d, %d, %d)", t, tr.op, tr.ro, tr.ri);
        if (!psi_of.count({tr.li, tr.ri})) return fail(OZ_ERR_ARG, "heff_plan_create: triple %d: no psi block (%d, %d)", t, tr.li, tr.ri);
        if (!psi_of.count({tr.lo, tr.ro})) return fail(OZ_ERR_ARG, "heff_plan_create: triple %d: no sigma block (%d, %d)", t, tr.lo, tr.ro);
        auto uk = std::make_tuple(tr.op, tr.lo, tr.li, tr.ri);
        auto it = u_of.find(uk);
        if (it == u_of.end()) {
            us.push_back(U{tr.op, tr.lo, tr.li, tr.ri, L_of[lk], psi_of[{tr.li, tr.ri}]});
            flops += 2.0 * ld[tr.lo] * ld[tr.li] * (p * rd[tr.ri]);
            it = u_of.emplace(uk, static_cast<int>(us.size()) - 1).first;
        }
        tri_u[t] = it->second;
        tri_R[t] = R_of[rk];
        tri_sigma[t] = psi_of[{tr.lo, tr.ro}];
        flops += 2.0 * (ld[tr.lo] * p) * rd[tr.ri] * rd[tr.ro];
        if (ld[tr.lo] * p > INT32_MAX / 2 || p * rd[tr.ri] > INT32_MAX / 2)
            return fail(OZ_ERR_ARG, "heff_plan_create: block too large");
        if (S && std::max<int64_t>(ld[tr.li], rd[tr.ri]) > max_exact_k(S, G))
            return fail(OZ_ERR_UNSUPPORTED, "heff_plan_create: inner dimension above the exact int32 range");
    }

    // Chunks: contiguous ranges of the triple list whose distinct first
    // products fit the T budget (FP64 values, and slices when emulated); a
    // first product used in two chunks is computed in both.  Within a chunk
    // the first products are ordered by psi block, then L block: the per-XCD
    // parts of the first phase's tile list then keep the products that read
    // one psi block together (1-3 % less time in that phase on the
    // block-sparse batch).  Results depend on neither the chunks nor the order.
    const size_t budget = ctx->heff_budget ? ctx->heff_budget : kHeffDefaultBudget;
    auto u_elems = [&](int u) { return ld[us[u].lo] * p * rd[us[u].ri]; };
    auto u_bytes = [&](int u) {
        const int64_t rows = ld[us[u].lo] * p, cols = rd[us[u].ri];
        return static_cast<size_t>(8 * rows * cols) +
               (S ? static_cast<size_t>(S) * round_up(rows, kRowQ) * round_up(cols, kKB) + 8 * round_up(rows, kRowQ) : 0);
    };
    struct HostChunk {
        int t0, t1;
        std::vector<int> us;        // global first-product indices
        std::vector<int64_t> t_off; // element offset of each in the shared T buffer
        int64_t t_total = 0;
    };
    std::vector<HostChunk> hc;
    {
        std::vector<char> in_chunk(us.size(), 0);
        size_t bytes = 0;
        HostChunk cur{0, 0, {}, {}, 0};
        for (int t = 0; t < n_triples; ++t) {
            const int u = tri_u[t];
            if (!in_chunk[u] && !cur.us.empty() && bytes + u_bytes(u) > budget) {
                cur.t1 = t;
                for (int x : cur.us) in_chunk[x] = 0;
                hc.push_back(cur);
                cur = HostChunk{t, t, {}, {}, 0};
                bytes = 0;
            }
            if (!in_chunk[u]) {
                in_chunk[u] = 1;
                cur.us.push_back(u);
                bytes += u_bytes(u);
            }
        }
        cur.t1 = n_triples;
        hc.push_back(cur);  // one chunk at least: it zeroes the sigma blocks no triple reaches
        for (auto &c : hc) {
            std::stable_sort(c.us.begin(), c.us.end(), [&](int a, int b) {
                return std::make_pair(us[a].psib, us[a].Lb) < std::make_pair(us[b].psib, us[b].Lb);
            });
            for (int u : c.us) {
                c.t_off.push_back(c.t_total);
                c.t_total += u_elems(u);
            }
        }
    }
    // sigma blocks per chunk: those with triples in it (continuing when an
    // earlier chunk had triples for them), and in the first chunk also the
    // blocks no triple reaches (zeroed)
    std::vector<int> n_trip(L->n_psi_blocks, 0);
    for (int t = 0; t < n_triples; ++t) ++n_trip[tri_sigma[t]];
    struct SigmaPart { int b; bool cont; std::vector<int> trips; };
    std::vector<std::vector<SigmaPart>> parts(hc.size());
    {
        std::vector<char> seen(L->n_psi_blocks, 0);
        for (size_t c = 0; c < hc.size(); ++c) {
            std::vector<std::vector<int>> by(L->n_psi_blocks);
            for (int t = hc[c].t0; t < hc[c].t1; ++t) by[tri_sigma[t]].push_back(t);
            for (int b = 0; b < L->n_psi_blocks; ++b) {
                if (!by[b].empty()) {
                    parts[c].push_back(SigmaPart{b, seen[b] != 0, by[b]});
                    seen[b] = 1;
                } else if (c == 0 && n_trip[b] == 0) {
                    parts[c].push_back(SigmaPart{b, false, {}});
                }
            }
        }
    }
    int64_t t_max = 1;
    for (auto &c : hc) t_max = std::max(t_max, c.t_total);

    hipError_t e;
    if ((e = hipSetDevice(ctx->device)) != hipSuccess) return hip_fail(e, "hipSetDevice");
    hipStream_t s = static_cast<hipStream_t>(stream);
    heff_plan P = new heff_plan_s();
    P->ctx = ctx;
    P->S = S;
    P->G = G;
    P->n = n;
    P->flops = flops;
    P->diag = diag;
    P->chunks.resize(hc.size());
    int rc = OZ_OK;
    void *mem = nullptr;
    if ((rc = alloc(P, sizeof(double) * t_max, &mem))) { free_plan(P); return rc; }
    P->T = static_cast<double *>(mem);
    P->T_bytes = sizeof(double) * t_max;

    if (S == 0) {
        for (size_t c = 0; c < hc.size(); ++c) {
            const HostChunk &h = hc[c];
            // tile edge per phase: 128, or 64 when the 128 tiles would not
            // give every compute unit two workgroups
            int64_t nL = 0, nR = 0;
            for (int u : h.us) nL += ceil_div(ld[us[u].lo], 128) * ceil_div(p * rd[us[u].ri], 128);
            for (const SigmaPart &sp : parts[c])
                nR += ceil_div(ld[L->psi_lr[2 * sp.b]] * p, 128) * ceil_div(rd[L->psi_lr[2 * sp.b + 1]], 128);
            const int bmL = dgemm_tile_for(nL, ctx->num_cu), bmR = dgemm_tile_for(nR, ctx->num_cu);
            const PairShape sh{bmL, bmL}, shR{bmR, bmR};
            // first product: T_u = L Psi  (op(B) = B, B offsets relative to psi)
            std::vector<Term64> termsL;
            std::vector<OutDesc> outsL;
            std::vector<std::vector<TileWork>> wl(h.us.size());
            for (size_t k = 0; k < h.us.size(); ++k) {
                const U &x = us[h.us[k]];
                const int64_t M = ld[x.lo], N = p * rd[x.ri], K = ld[x.li];
                Term64 tm{};
                tm.A = L_data + L->L_offset[x.Lb];
                tm.lda = K;
                tm.B = reinterpret_cast<const double *>(static_cast<intptr_t>(L->psi_offset[x.psib]));
                tm.ldb = N;
                tm.K = static_cast<int32_t>(K);
                tm.alpha = 1.0;
                termsL.push_back(tm);
                outsL.push_back(OutDesc{P->T + h.t_off[k], N, static_cast<int32_t>(M), static_cast<int32_t>(N)});
                walk_output(M, N, sh, [&](int64_t m0, int64_t n0) {
                    return TileWork{TileDesc{static_cast<int32_t>(k), static_cast<int32_t>(k + 1), static_cast<int32_t>(m0),
                                             static_cast<int32_t>(n0), static_cast<int32_t>(k), 0}, K};
                }, &wl[k]);
            }
            // second product: sigma' (+)= sum alpha T'_u R^T  (op(B) = R^T)
            std::vector<int> local(us.size(), -1);
            for (size_t k = 0; k < h.us.size(); ++k) local[h.us[k]] = static_cast<int>(k);
            std::vector<Term64> termsR;
            std::vector<OutDesc> outsR;
            std::vector<std::vector<TileWork>> wr(parts[c].size());
            for (size_t q = 0; q < parts[c].size(); ++q) {
                const SigmaPart &sp = parts[c][q];
                const int lo = L->psi_lr[2 * sp.b], ro = L->psi_lr[2 * sp.b + 1];
                const int64_t M = ld[lo] * p, N = rd[ro];
                const int tb = static_cast<int>(termsR.size());
                int64_t cost = 0;
                for (int t : sp.trips) {
                    const int k = local[tri_u[t]];
                    const U &x = us[tri_u[t]];
                    Term64 tm{};
                    tm.A = P->T + h.t_off[k];
                    tm.lda = rd[x.ri];
                    tm.B = R_data + L->R_offset[tri_R[t]];
                    tm.ldb = rd[x.ri];
                    tm.K = static_cast<int32_t>(rd[x.ri]);
                    tm.alpha = triples[t].alpha;
                    termsR.push_back(tm);
                    cost += rd[x.ri];
                }
                const int te = static_cast<int>(termsR.size());
                OutDesc o{reinterpret_cast<double *>(static_cast<intptr_t>(L->psi_offset[sp.b])), N,
                          static_cast<int32_t>(M), static_cast<int32_t>(N)};
                o.cont = sp.cont ? 1 : 0;
                outsR.push_back(o);
                walk_output(M, N, shR, [&](int64_t m0, int64_t n0) {
                    return TileWork{TileDesc{tb, te, static_cast<int32_t>(m0), static_cast<int32_t>(n0), static_cast<int32_t>(q), 0},
                                    cost + 1};
                }, &wr[q]);
            }
            std::vector<TileDesc> tl, tr;
            std::vector<int64_t> cl, cr;
            xcd_order(wl, &tl, &cl);
            xcd_order(wr, &tr, &cr);
            TileDesc *dt;
            Term64 *dm;
            OutDesc *dout;
            HeffChunk &ch = P->chunks[c];
            if ((rc = upload(P, tl, &dt)) || (rc = upload(P, termsL, &dm)) || (rc = upload(P, outsL, &dout))) { free_plan(P); return rc; }
            ch.d64L.tiles = dt; ch.d64L.terms = dm; ch.d64L.outs = dout;
            ch.d64L.ntiles = static_cast<int32_t>(tl.size());
            ch.d64L.mode = kModeGemm;
            ch.d64L.tile = bmL;
            if ((rc = upload(P, tr, &dt)) || (rc = upload(P, termsR, &dm)) || (rc = upload(P, outsR, &dout))) { free_plan(P); return rc; }
            ch.d64R.tiles = dt; ch.d64R.terms = dm; ch.d64R.outs = dout;
            ch.d64R.ntiles = static_cast<int32_t>(tr.size());
            ch.d64R.mode = kModeAccum;
            ch.d64R.tile = bmR;
        }
        *out = P;
        return OZ_OK;
    }

    // ---- emulated path: slice every L and R block once ----
    SliceSet Ls, Rs;
    std::vector<int64_t> L_eoff(L->n_L_blocks), L_poff(L->n_L_blocks), R_eoff(L->n_R_blocks), R_poff(L->n_R_blocks);
    for (int i = 0; i < L->n_L_blocks; ++i) {
        const int lo = L->L_key[3 * i + 1], li = L->L_key[3 * i + 2];
        Ls.add(L->L_offset[i], ld[li], ld[lo], ld[li], false, S, &L_eoff[i], &L_poff[i]);
    }
    for (int i = 0; i < L->n_R_blocks; ++i) {
        const int ro = L->R_key[3 * i + 1], ri = L->R_key[3 * i + 2];
        Rs.add(L->R_offset[i], rd[ri], rd[ro], rd[ri], false, S, &R_eoff[i], &R_poff[i]);
    }
    int32_t *Le, *Re;
    int8_t *Lp, *Rp;
    if ((rc = slice_once(P, Ls, L_data, S, s, &Le, &Lp)) || (rc = slice_once(P, Rs, R_data, S, s, &Re, &Rp))) { free_plan(P); return rc; }

    // psi blocks sliced by columns of the left x (phys * right) view, on every apply
    SliceSet Ps;
    Ps.split_cols = true;  // row chunks of long columns in parallel, combined through codes
    std::vector<int64_t> P_eoff(L->n_psi_blocks), P_poff(L->n_psi_blocks);
    for (int b = 0; b < L->n_psi_blocks; ++b) {
        const int l = L->psi_lr[2 * b], r = L->psi_lr[2 * b + 1];
        Ps.add(L->psi_offset[b], p * rd[r], p * rd[r], ld[l], true, S, &P_eoff[b], &P_poff[b]);
    }
    if ((rc = upload(P, Ps.blocks, &P->psi_blocks)) || (rc = upload(P, Ps.etasks, &P->psi_etasks)) ||
        (rc = upload(P, Ps.stasks, &P->psi_stasks))) { free_plan(P); return rc; }
    void *pe, *pp;
    if ((rc = alloc(P, sizeof(int32_t) * std::max<int64_t>(Ps.e_total, 1), &pe)) ||
        (rc = alloc(P, std::max<int64_t>(Ps.p_total, 256), &pp))) { free_plan(P); return rc; }
    P->n_psi_etasks = static_cast<int>(Ps.etasks.size());
    P->n_psi_stasks = static_cast<int>(Ps.stasks.size());
    P->psi_e = static_cast<int32_t *>(pe);
    P->psi_p = static_cast<int8_t *>(pp);
    if (Ps.e_total > 0) {
        const std::vector<int32_t> init(static_cast<size_t>(Ps.e_total), kEmaxZero);
        if ((rc = upload(P, init, &P->psi_emax))) { free_plan(P); return rc; }
        P->psi_e_total = Ps.e_total;
    }

    // per chunk: T_u sliced by rows of the (left * phys) x right view into the
    // shared slice buffer; the terms and outputs of both phases
    struct HostLists {
        SliceSet Ts;
        std::vector<int64_t> T_eoff, T_poff;
        std::vector<TermDesc> termsL, termsR;
        std::vector<OutDesc> outsL, outsR;
        std::vector<int> sigma_tb, sigma_te;
        std::vector<int64_t> sigma_cost;
    };
    std::vector<HostLists> hl(hc.size());
    int64_t Te_max = 1, Tp_max = 256;
    for (size_t c = 0; c < hc.size(); ++c) {
        const HostChunk &h = hc[c];
        HostLists &x = hl[c];
        x.T_eoff.resize(h.us.size());
        x.T_poff.resize(h.us.size());
        for (size_t k = 0; k < h.us.size(); ++k) {
            const U &u = us[h.us[k]];
            x.Ts.add(h.t_off[k], rd[u.ri], ld[u.lo] * p, rd[u.ri], false, S, &x.T_eoff[k], &x.T_poff[k]);
        }
        Te_max = std::max(Te_max, x.Ts.e_total);
        Tp_max = std::max(Tp_max, x.Ts.p_total);
    }
    void *te_, *tp;
    if ((rc = alloc(P, sizeof(int32_t) * Te_max, &te_)) || (rc = alloc(P, Tp_max, &tp))) { free_plan(P); return rc; }
    P->T_e = static_cast<int32_t *>(te_);
    P->T_p = static_cast<int8_t *>(tp);
    P->T_bytes += sizeof(int32_t) * Te_max + Tp_max;
    // T's row exponents from its producer when every row of the (left * phys)
    // x right view takes whole 32-column groups of the first product (phys =
    // 1, or right dimensions that are multiples of 32): the first phase's
    // epilogue leaves exponent-code maxima in T_emax and a small kernel turns
    // them into T_e, instead of a pass that reads T.
    bool any_fuse = false;
    for (size_t c = 0; c < hc.size(); ++c) {
        bool f = hl[c].Ts.e_total > 0;
        for (int u : hc[c].us) f = f && (p == 1 || rd[us[u].ri] % 32 == 0);
        P->chunks[c].fuse_T = f;
        any_fuse = any_fuse || f;
    }
    const std::vector<int32_t> emax_init(static_cast<size_t>(Te_max), kEmaxZero);
    if (any_fuse && (rc = upload(P, emax_init, &P->T_emax))) { free_plan(P); return rc; }

    for (size_t c = 0; c < hc.size(); ++c) {
        const HostChunk &h = hc[c];
        HostLists &x = hl[c];
        HeffChunk &ch = P->chunks[c];
        ch.T_e_total = x.Ts.e_total;
        ch.n_T_etasks = static_cast<int>(x.Ts.etasks.size());
        ch.n_T_stasks = static_cast<int>(x.Ts.stasks.size());
        if ((rc = upload(P, x.Ts.blocks, &ch.T_blocks)) || (rc = upload(P, x.Ts.etasks, &ch.T_etasks)) ||
            (rc = upload(P, x.Ts.stasks, &ch.T_stasks))) { free_plan(P); return rc; }
        std::vector<int> local(us.size(), -1);
        for (size_t k = 0; k < h.us.size(); ++k) {
            local[h.us[k]] = static_cast<int>(k);
            const U &u = us[h.us[k]];
            const int64_t M = ld[u.lo], N = p * rd[u.ri], K = ld[u.li];
            TermDesc tm{};
            tm.A = Lp + L_poff[u.Lb];
            tm.e = Le + L_eoff[u.Lb];
            tm.a_rows_p = round_up(M, kRowQ);
            tm.B = P->psi_p + P_poff[u.psib];
            tm.f = P->psi_e + P_eoff[u.psib];
            tm.b_rows_p = round_up(N, kRowQ);
            tm.kblocks = static_cast<int32_t>(ceil_div(K, kKB));
            tm.alpha = 1.0;
            x.termsL.push_back(tm);
            OutDesc o{P->T + h.t_off[k], N, static_cast<int32_t>(M), static_cast<int32_t>(N)};
            if (ch.fuse_T) {
                o.emax = P->T_emax + x.T_eoff[k];
                o.ep = static_cast<int32_t>(p);
                o.en = static_cast<int32_t>(rd[u.ri]);
            }
            x.outsL.push_back(o);
        }
        for (const SigmaPart &sp : parts[c]) {
            const int lo = L->psi_lr[2 * sp.b], ro = L->psi_lr[2 * sp.b + 1];
            const int64_t M = ld[lo] * p, N = rd[ro];
            x.sigma_tb.push_back(static_cast<int>(x.termsR.size()));
            int64_t cost = 0;
            for (int t : sp.trips) {
                const int k = local[tri_u[t]];
                const U &u = us[tri_u[t]];
                TermDesc tm{};
                tm.A = P->T_p + x.T_poff[k];
                tm.e = P->T_e + x.T_eoff[k];
                tm.a_rows_p = round_up(M, kRowQ);
                tm.B = Rp + R_poff[tri_R[t]];
                tm.f = Re + R_eoff[tri_R[t]];
                tm.b_rows_p = round_up(N, kRowQ);
                tm.kblocks = static_cast<int32_t>(ceil_div(rd[u.ri], kKB));
                tm.alpha = triples[t].alpha;
                x.termsR.push_back(tm);
                cost += tm.kblocks;
            }
            x.sigma_te.push_back(static_cast<int>(x.termsR.size()));
            x.sigma_cost.push_back(cost);
            OutDesc o{reinterpret_cast<double *>(static_cast<intptr_t>(L->psi_offset[sp.b])), N,
                      static_cast<int32_t>(M), static_cast<int32_t>(N)};
            o.cont = sp.cont ? 1 : 0;
            x.outsR.push_back(o);
        }
        TermDesc *dmL, *dmR;
        OutDesc *doL, *doR;
        if ((rc = upload(P, x.termsL, &dmL)) || (rc = upload(P, x.outsL, &doL)) || (rc = upload(P, x.termsR, &dmR)) ||
            (rc = upload(P, x.outsR, &doR))) { free_plan(P); return rc; }
        ch.argsL.terms = dmL; ch.argsL.outs = doL; ch.argsL.mode = kModeGemm;
        ch.argsR.terms = dmR; ch.argsR.outs = doR; ch.argsR.mode = kModeAccum;
        // tile counters of the streamed launches (zero; every launch leaves them zero)
        const std::vector<int32_t> zq(kStreamQueueInts, 0);
        if ((rc = upload(P, zq, &ch.argsL.queue)) || (rc = upload(P, zq, &ch.argsR.queue))) { free_plan(P); return rc; }
    }

    // tile lists of chunk c per variant, in order 0 (XCD parts of equal
    // cost), 1 (longest tile first) or 2 (whole outputs to XCDs, heaviest
    // first to the least loaded)
    auto tiles_for = [&](size_t c, int v, int order, std::vector<TileDesc> *tl, std::vector<TileDesc> *tr,
                         std::vector<int64_t> *cl, std::vector<int64_t> *cr) {
        const HostLists &x = hl[c];
        const PairShape sh = pair_shape(S, G, v);
        std::vector<std::vector<TileWork>> wl(x.outsL.size()), wr(x.outsR.size());
        for (size_t u = 0; u < x.outsL.size(); ++u) {
            const OutDesc &o = x.outsL[u];
            const int64_t cst = static_cast<int64_t>(x.termsL[u].kblocks) * sh.bm * sh.bn;
            walk_output(o.M, o.N, sh, [&](int64_t m0, int64_t n0) {
                return TileWork{TileDesc{static_cast<int32_t>(u), static_cast<int32_t>(u + 1), static_cast<int32_t>(m0),
                                         static_cast<int32_t>(n0), static_cast<int32_t>(u), 0}, cst};
            }, &wl[u]);
        }
        for (size_t q = 0; q < x.outsR.size(); ++q) {
            const OutDesc &o = x.outsR[q];
            const int64_t cst = (x.sigma_cost[q] + 1) * sh.bm * sh.bn;
            walk_output(o.M, o.N, sh, [&](int64_t m0, int64_t n0) {
                return TileWork{TileDesc{x.sigma_tb[q], x.sigma_te[q], static_cast<int32_t>(m0), static_cast<int32_t>(n0),
                                         static_cast<int32_t>(q), 0}, cst};
            }, &wr[q]);
        }
        if (order == 0) {
            xcd_order(wl, tl, cl);
            xcd_order(wr, tr, cr);
        } else if (order == 1) {
            longest_first(wl, tl, cl);
            longest_first(wr, tr, cr);
        } else {
            output_lpt_order(wl, tl, cl);
            output_lpt_order(wr, tr, cr);
        }
    };

    const int fixed = ctx->variant[S][G];
    std::vector<int> cands;
    for (int v = 0; v < pair_num_variants(); ++v)
        if (pair_variant_ok(G, v) && (fixed < 0 ? (ctx->autotune || v == pair_default_variant(G)) : v == fixed))
            cands.push_back(v);
    // Autotuning on the first chunk: time each candidate (tile variant, tile
    // order, launch) on its whole tile list or an even sample of it, scaled
    // by the sample's share of the total cost; inputs are zeroed scratch (the
    // timing does not depend on the values).  Every chunk then uses the
    // choice per phase.
    double bestL = -1, bestR = -1;
    void *tmp_sigma = nullptr;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    // both phases fixed by the context: nothing is timed
    const bool fixed_phases = ctx->heff_fix[0][0] >= 0 && ctx->heff_fix[1][0] >= 0;
    if (fixed_phases && (!pair_variant_ok(G, ctx->heff_fix[0][0]) || !pair_variant_ok(G, ctx->heff_fix[1][0]))) {
        free_plan(P);
        return fail(OZ_ERR_ARG, "heff_plan_create: fixed tile variant not built for ndiag %d", G);
    }
    const bool tuning = !fixed_phases && (cands.size() > 1 || ctx->autotune);
    if (tuning) {
        if ((e = hipMalloc(&tmp_sigma, sizeof(double) * std::max<int64_t>(n, 1))) != hipSuccess) { free_plan(P); return hip_fail(e, "heff_plan_create: tuning buffer"); }
        hipMemsetAsync(P->psi_p, 0, std::max<int64_t>(Ps.p_total, 256), s);
        hipMemsetAsync(P->psi_e, 0, sizeof(int32_t) * std::max<int64_t>(Ps.e_total, 1), s);
        hipMemsetAsync(P->T_p, 0, Tp_max, s);
        hipMemsetAsync(P->T_e, 0, sizeof(int32_t) * Te_max, s);
        if ((e = hipEventCreate(&ev0)) != hipSuccess || (e = hipEventCreate(&ev1)) != hipSuccess) {
            if (ev0) hipEventDestroy(ev0);
            hipFree(tmp_sigma);
            free_plan(P);
            return hip_fail(e, "heff_plan_create: tuning events");
        }
    }
    // Candidates: tile variant x tile order (the XCD order first, the
    // default) x launch: one workgroup per tile; the streamed kernel, whose
    // resident workgroups take tiles from counters and prefetch across
    // items; the resident kernel on a precomputed schedule (first phase
    // only, for the variants it is built for), which streams the K blocks
    // of consecutive tiles through one ring; or the paired-term kernel
    // (second phase only, 64 x 64 tiles), eight waves per tile taking two
    // terms at a time.
    struct Run { int v; int order; int kind; int cus; };  // kind 0 per tile, 1 streamed (cus), 2 resident, 3 paired terms
    constexpr double kStreamMaxMeanBlocks = 16.0;
    const int forced = ctx->heff_launch;  // -1 timed, 0 per tile, k > 0 streamed, resident or paired terms
    const int stream_cus_of = forced > 0 ? std::min(forced, ctx->num_cu) : ctx->num_cu;
    // the launches a phase may use for variant v
    auto kinds_for = [&](int ph, int v) {
        std::vector<int> k;
        if (forced == kHeffLaunchResident) {
            k.push_back(ph == 0 && pair_resident_per_cu(S, G, v) > 0 ? 2 : 0);
        } else if (forced == kHeffLaunchPairedTerms) {
            k.push_back(ph == 1 && pair_terms2_ok(S, G, v) ? 3 : 0);
        } else if (forced >= 0) {
            k.push_back(forced > 0 ? 1 : 0);
        } else {
            k.push_back(0);
            if (tuning && ph == 0) {
                k.push_back(1);
                if (pair_resident_per_cu(S, G, v) > 0) k.push_back(2);
            }
            if (tuning && ph == 1 && pair_terms2_ok(S, G, v)) k.push_back(3);
        }
        return k;
    };
    Run chosenL{cands.front(), 0, 0, 0}, chosenR{cands.front(), 0, 0, 0};
    {
        const std::vector<int> kl = kinds_for(0, chosenL.v), kr = kinds_for(1, chosenR.v);
        chosenL.kind = kl.front();
        chosenR.kind = kr.front();
        chosenL.cus = chosenL.kind == 1 ? stream_cus_of : 0;
        chosenR.cus = chosenR.kind == 1 ? stream_cus_of : 0;
    }
    // Timing sample: the equivalent of 64 tiles of 16 K blocks per CU, at
    // least 8 and at most 64 tiles per CU, as 8 windows of consecutive list
    // positions spread evenly over the list.  A window keeps the XCD order's
    // placement and the operand reuse between neighbouring tiles that the
    // orders differ in; the spread samples a longest-first list at every
    // length.
    const size_t cap = static_cast<size_t>(64) * ctx->num_cu;
    const size_t floor_tiles = static_cast<size_t>(8) * ctx->num_cu;
    TileDesc *tmp_tiles = nullptr;
    int32_t *tmp_off = nullptr;
    // the tuning's scratch buffers and events, released on every path
    auto free_tuning = [&]() {
        if (tmp_sigma) hipFree(tmp_sigma);
        if (tmp_tiles) hipFree(tmp_tiles);
        if (tmp_off) hipFree(tmp_off);
        if (ev0) hipEventDestroy(ev0);
        if (ev1) hipEventDestroy(ev1);
        tmp_sigma = nullptr;
        tmp_tiles = nullptr;
        tmp_off = nullptr;
        ev0 = ev1 = nullptr;
    };
    if (tuning && ((e = hipMalloc(&tmp_tiles, sizeof(TileDesc) * (cap + 8))) != hipSuccess ||
                   (e = hipMalloc(&tmp_off, sizeof(int32_t) * (static_cast<size_t>(kMaxResidentPerCu) * ctx->num_cu + 1))) != hipSuccess)) {
        free_tuning();
        free_plan(P);
        return hip_fail(e, "heff_plan_create: tuning buffer");
    }
    if (fixed_phases) {
        for (int ph = 0; ph < 2; ++ph) {
            const int l = ctx->heff_fix[ph][2];
            Run &r = ph == 0 ? chosenL : chosenR;
            r = Run{ctx->heff_fix[ph][0], ctx->heff_fix[ph][1], 0, 0};
            if (l == kHeffLaunchResident) {
                if (ph != 0 || pair_resident_per_cu(S, G, r.v) <= 0) {
                    free_plan(P);
                    return fail(OZ_ERR_ARG, "heff_plan_create: resident launch not built for phase %d, variant %d", ph, r.v);
                }
                r.kind = 2;
            } else if (l == kHeffLaunchPairedTerms) {
                if (ph != 1 || !pair_terms2_ok(S, G, r.v)) {
                    free_plan(P);
                    return fail(OZ_ERR_ARG, "heff_plan_create: paired-term launch not built for phase %d, variant %d", ph, r.v);
                }
                r.kind = 3;
            } else if (l > 0) {
                r.kind = 1;
                r.cus = std::min(l, ctx->num_cu);
            }
        }
    } else if (tuning) {
        std::vector<TileDesc> tl, tr, sample, perm;
        std::vector<int64_t> cl, cr, scost;
        std::vector<int32_t> off;
        for (int v : cands)
            for (int order : {0, 1, 2}) {
                tiles_for(0, v, order, &tl, &tr, &cl, &cr);
                for (int ph = 0; ph < 2; ++ph) {
                    const std::vector<int64_t> &cost = ph == 0 ? cl : cr;
                    const std::vector<TileDesc> &list = ph == 0 ? tl : tr;
                    int64_t total = 0, items = 0;
                    for (auto cc : cost) {
                        total += cc;
                        items += cc > 0;
                    }
                    const PairShape shp = pair_shape(S, G, v);
                    const double blocks_per_tile = items ? static_cast<double>(total) / items / (shp.bm * shp.bn) : 1.0;
                    // the timing sample (the whole list when it is short)
                    const size_t n_sample = std::min(cap, std::max(floor_tiles, static_cast<size_t>(16.0 * cap / std::max(blocks_per_tile, 1.0))));
                    int64_t part = 0;
                    sample.clear();
                    scost.clear();
                    if (list.size() <= n_sample) {
                        sample = list;
                        scost = cost;
                        part = total;
                    } else {
                        constexpr size_t kWindows = 8;
                        const size_t wlen = std::max<size_t>(n_sample / kWindows / 8 * 8, 8);
                        for (size_t w = 0; w < kWindows; ++w) {
                            const size_t start = (w * list.size() / kWindows) / 8 * 8;
                            for (size_t j = start; j < std::min(start + wlen, list.size()); ++j) {
                                sample.push_back(list[j]);
                                scost.push_back(cost[j]);
                                part += cost[j];
                            }
                        }
                    }
                    for (int kind : kinds_for(ph, v)) {
                        // Timed choice: the streamed kernel saves a fixed cost
                        // per (tile, term) item (the first K block's load, the
                        // exposed epilogue), so it is a candidate for the
                        // GEMM-mode phase with short items only; in the
                        // accumulating phase it was slower at every measured
                        // shape.
                        if (kind == 1 && forced < 0 && (ph == 1 || blocks_per_tile > kStreamMaxMeanBlocks)) continue;
                        PairArgs a = ph == 0 ? P->chunks[0].argsL : P->chunks[0].argsR;
                        a.stream_cus = kind == 1 ? stream_cus_of : 0;
                        a.nwg = 0;
                        a.wg_off = nullptr;
                        a.terms2 = kind == 3 ? 1 : 0;
                        const std::vector<TileDesc> *up = &sample;
                        if (kind == 2) {
                            const int nwg = std::min(pair_resident_per_cu(S, G, v), kMaxResidentPerCu) * ctx->num_cu;
                            resident_schedule(sample, scost, nwg, resident_start_cost(shp), &perm, &off);
                            if ((e = hipMemcpy(tmp_off, off.data(), sizeof(int32_t) * off.size(), hipMemcpyHostToDevice)) != hipSuccess) {
                                free_tuning();
                                free_plan(P);
                                return hip_fail(e, "heff_plan_create: tuning schedule");
                            }
                            a.nwg = nwg;
                            a.wg_off = tmp_off;
                            up = &perm;
                        }
                        if (up->empty()) continue;
                        if ((e = hipMemcpy(tmp_tiles, up->data(), sizeof(TileDesc) * up->size(), hipMemcpyHostToDevice)) != hipSuccess) {
                            free_tuning();
                            free_plan(P);
                            return hip_fail(e, "heff_plan_create: tuning sample");
                        }
                        a.tiles = tmp_tiles;
                        a.ntiles = static_cast<int32_t>(up->size());
                        if (ph == 1) a.out_base = static_cast<double *>(tmp_sigma);
                        // a warm-up launch, then the faster of two timed ones
                        float ms = 0.f;
                        for (int rep = 0; rep < 3; ++rep) {
                            float r = 0.f;
                            hipEventRecord(ev0, s);
                            if ((e = launch_pair_grouped(S, G, v, a, s)) != hipSuccess) {
                                free_tuning();
                                free_plan(P);
                                return hip_fail(e, "heff_plan_create: tuning launch");
                            }
                            hipEventRecord(ev1, s);
                            hipEventSynchronize(ev1);
                            hipEventElapsedTime(&r, ev0, ev1);
                            if (rep == 1 || (rep > 1 && r < ms)) ms = r;
                        }
                        const double est = part > 0 ? ms * static_cast<double>(total) / static_cast<double>(part) : 0.0;
                        double &best = ph == 0 ? bestL : bestR;
                        if (best < 0 || est < best) {
                            best = est;
                            (ph == 0 ? chosenL : chosenR) = Run{v, order, kind, kind == 1 ? stream_cus_of : 0};
                        }
                    }
                }
            }
        hipStreamSynchronize(s);
        free_tuning();
        // the timed launches of the first phase may have left maxima
        if (P->T_emax && (e = hipMemcpy(P->T_emax, emax_init.data(), sizeof(int32_t) * emax_init.size(),
                                        hipMemcpyHostToDevice)) != hipSuccess) { free_plan(P); return hip_fail(e, "heff_plan_create: reset"); }
    }
    // every chunk: the chosen tile lists, schedules and launches per phase
    for (size_t c = 0; c < hc.size(); ++c) {
        std::vector<TileDesc> l1, r1, l2, r2;
        std::vector<int64_t> cl1, cr1, cl2, cr2;
        tiles_for(c, chosenL.v, chosenL.order, &l1, &r1, &cl1, &cr1);
        tiles_for(c, chosenR.v, chosenR.order, &l2, &r2, &cl2, &cr2);
        HeffChunk &ch = P->chunks[c];
        for (int ph = 0; ph < 2; ++ph) {
            const Run &run = ph == 0 ? chosenL : chosenR;
            const std::vector<TileDesc> &list = ph == 0 ? l1 : r2;
            const std::vector<int64_t> &cost = ph == 0 ? cl1 : cr2;
            PairArgs &a = ph == 0 ? ch.argsL : ch.argsR;
            a.stream_cus = run.kind == 1 ? run.cus : 0;
            a.nwg = 0;
            a.wg_off = nullptr;
            a.terms2 = run.kind == 3 ? 1 : 0;
            TileDesc *d = nullptr;
            if (run.kind == 2) {
                const int nwg = std::min(pair_resident_per_cu(S, G, run.v), kMaxResidentPerCu) * ctx->num_cu;
                std::vector<TileDesc> perm;
                std::vector<int32_t> off;
                resident_schedule(list, cost, nwg, resident_start_cost(pair_shape(S, G, run.v)), &perm, &off);
                int32_t *doff = nullptr;
                if ((rc = upload(P, perm, &d)) || (rc = upload(P, off, &doff))) { free_plan(P); return rc; }
                a.tiles = d;
                a.ntiles = static_cast<int32_t>(perm.size());
                a.nwg = nwg;
                a.wg_off = doff;
            } else {
                if ((rc = upload(P, list, &d))) { free_plan(P); return rc; }
                a.tiles = d;
                a.ntiles = static_cast<int32_t>(list.size());
            }
        }
    }
    P->varL = chosenL.v;
    P->varR = chosenR.v;
    P->choice[0][0] = chosenL.v;
    P->choice[0][1] = chosenL.order;
    auto launch_code = [](const Run &r) {
        return r.kind == 2 ? kHeffLaunchResident : r.kind == 3 ? kHeffLaunchPairedTerms : r.cus;
    };
    P->choice[0][2] = launch_code(chosenL);
    P->choice[1][0] = chosenR.v;
    P->choice[1][1] = chosenR.order;
    P->choice[1][2] = launch_code(chosenR);
    if ((e = hipStreamSynchronize(s)) != hipSuccess) { free_plan(P); return hip_fail(e, "heff_plan_create: sync"); }
    *out = P;
    return OZ_OK;
}

namespace {

// The launches of one apply, in order, on stream s.
int enqueue_apply(heff_plan P, const double *psi, double *sigma, hipStream_t s) {
    ozaki_ctx ctx = P->ctx;
    hipError_t e;
    if (P->S == 0) {
        for (const HeffChunk &ch : P->chunks) {
            hipEvent_t t0 = mark(ctx, s);
            Dgemm64Args a = ch.d64L;
            a.b_base = psi;
            if ((e = launch_dgemm_grouped(false, a, s)) != hipSuccess) return hip_fail(e, "heff_apply: first product");
            hipEvent_t t1 = mark(ctx, s);
            phase(ctx, OZ_PHASE_HEFF_L, t0, t1);
            Dgemm64Args b = ch.d64R;
            b.out_base = sigma;
            if ((e = launch_dgemm_grouped(true, b, s)) != hipSuccess) return hip_fail(e, "heff_apply: second product");
            hipEvent_t t2 = mark(ctx, s);
            phase(ctx, OZ_PHASE_HEFF_R, t1, t2);
        }
    } else {
        hipEvent_t t0 = mark(ctx, s);
        if ((e = launch_exponents_grouped(P->psi_blocks, P->psi_etasks, P->n_psi_etasks, psi, P->psi_e, ctx->d_flags, s, P->psi_emax)) != hipSuccess ||
            (e = launch_emax_finish(P->psi_emax, P->psi_e, P->psi_e_total, ctx->d_flags, s)) != hipSuccess ||
            (e = launch_slice_grouped(P->S, P->psi_blocks, P->psi_stasks, P->n_psi_stasks, psi, P->psi_e, P->psi_p, s)) != hipSuccess)
            return hip_fail(e, "heff_apply: slicing psi");
        hipEvent_t t1 = mark(ctx, s);
        phase(ctx, OZ_PHASE_HEFF_AUX, t0, t1);
        for (const HeffChunk &ch : P->chunks) {
            hipEvent_t c0 = mark(ctx, s);
            if ((e = launch_pair_grouped(P->S, P->G, P->varL, ch.argsL, s)) != hipSuccess) return hip_fail(e, "heff_apply: first product");
            hipEvent_t c1 = mark(ctx, s);
            phase(ctx, OZ_PHASE_HEFF_L, c0, c1);
            if ((e = ch.fuse_T ? launch_emax_finish(P->T_emax, P->T_e, ch.T_e_total, ctx->d_flags, s)
                               : launch_exponents_grouped(ch.T_blocks, ch.T_etasks, ch.n_T_etasks, P->T, P->T_e, ctx->d_flags, s)) != hipSuccess ||
                (e = launch_slice_grouped(P->S, ch.T_blocks, ch.T_stasks, ch.n_T_stasks, P->T, P->T_e, P->T_p, s)) != hipSuccess)
                return hip_fail(e, "heff_apply: slicing T");
            hipEvent_t c2 = mark(ctx, s);
            phase(ctx, OZ_PHASE_HEFF_AUX, c1, c2);
            PairArgs b = ch.argsR;
            b.out_base = sigma;
            if ((e = launch_pair_grouped(P->S, P->G, P->varR, b, s)) != hipSuccess) return hip_fail(e, "heff_apply: second product");
            hipEvent_t c3 = mark(ctx, s);
            phase(ctx, OZ_PHASE_HEFF_R, c2, c3);
        }
    }
    if (P->diag) {
        if ((e = launch_diag_axpy(P->diag, psi, sigma, P->n, s)) != hipSuccess) return hip_fail(e, "heff_apply: diagonal");
    }
    return OZ_OK;
}

constexpr size_t kMaxGraphs = 96;

// Capture the apply sequence for (psi, sigma) and instantiate it; evicts the
// least recently used graph when the cache is full.
int capture_apply(heff_plan P, const double *psi, double *sigma, hipStream_t s,
                  heff_plan_s::GraphSlot **out) {
    hipError_t e;
    if (!P->cap && (e = hipStreamCreateWithFlags(&P->cap, hipStreamNonBlocking)) != hipSuccess)
        return hip_fail(e, "heff_apply: capture stream");
    if (P->graphs.size() >= kMaxGraphs) {
        size_t lru = 0;
        for (size_t i = 1; i < P->graphs.size(); ++i)
            if (P->graphs[i].used < P->graphs[lru].used) lru = i;
        // the evicted graph may still run on the caller's stream
        if ((e = hipStreamSynchronize(s)) != hipSuccess) return hip_fail(e, "heff_apply: sync before eviction");
        hipGraphExecDestroy(P->graphs[lru].exec);
        P->graphs.erase(P->graphs.begin() + static_cast<std::ptrdiff_t>(lru));
    }
    if ((e = hipStreamBeginCapture(P->cap, hipStreamCaptureModeThreadLocal)) != hipSuccess)
        return hip_fail(e, "heff_apply: begin capture");
    const int rc = enqueue_apply(P, psi, sigma, P->cap);
    hipGraph_t graph = nullptr;
    e = hipStreamEndCapture(P->cap, &graph);
    if (rc != OZ_OK) {
        if (graph) hipGraphDestroy(graph);
        return rc;
    }
    if (e != hipSuccess) return hip_fail(e, "heff_apply: end capture");
    hipGraphExec_t exec = nullptr;
    e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    hipGraphDestroy(graph);
    if (e != hipSuccess) return hip_fail(e, "heff_apply: instantiate");
    P->graphs.push_back({psi, sigma, exec, 0});
    *out = &P->graphs.back();
    return OZ_OK;
}

}  // namespace

int heff_apply(heff_plan P, const double *psi, double *sigma, void *stream) {
    if (!P) return fail(OZ_ERR_ARG, "heff_apply: plan is NULL");
    if (P->n > 0 && (!psi || !sigma)) return fail(OZ_ERR_ARG, "heff_apply: psi / sigma NULL");
    if (P->n > 0) {
        const uintptr_t a = reinterpret_cast<uintptr_t>(psi), b = reinterpret_cast<uintptr_t>(sigma);
        const uintptr_t bytes = static_cast<uintptr_t>(P->n) * sizeof(double);
        if (a < b + bytes && b < a + bytes) return fail(OZ_ERR_ARG, "heff_apply: psi and sigma overlap");
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    ozaki_ctx ctx = P->ctx;
    hipError_t e;
    if ((e = hipSetDevice(ctx->device)) != hipSuccess) return hip_fail(e, "hipSetDevice");
    if (P->n == 0) return OZ_OK;
    // replay a captured graph unless phases are being timed or the caller's
    // stream is itself being captured (then the launches go into that graph)
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if ((e = hipStreamIsCapturing(s, &cs)) != hipSuccess) return hip_fail(e, "heff_apply: capture status");
    if (!P->use_graphs || ctx->timing || cs != hipStreamCaptureStatusNone) return enqueue_apply(P, psi, sigma, s);
    heff_plan_s::GraphSlot *g = nullptr;
    for (auto &x : P->graphs)
        if (x.psi == psi && x.sigma == sigma) g = &x;
    if (!g) {
        const int rc = capture_apply(P, psi, sigma, s, &g);
        if (rc != OZ_OK) return rc;
    }
    g->used = ++P->clock;
    if ((e = hipGraphLaunch(g->exec, s)) != hipSuccess) return hip_fail(e, "heff_apply: graph launch");
    return OZ_OK;
}

int heff_plan_set_graphs(heff_plan P, int enable) {
    if (!P) return fail(OZ_ERR_ARG, "heff_plan_set_graphs: plan is NULL");
    P->use_graphs = enable != 0;
    return OZ_OK;
}

int heff_plan_graph_count(heff_plan P) {
    if (!P) return fail(OZ_ERR_ARG, "heff_plan_graph_count: plan is NULL");
    return static_cast<int>(P->graphs.size());
}

int64_t heff_vector_length(heff_plan P) { return P ? P->n : -1; }

int heff_plan_variants(heff_plan P, int32_t *first, int32_t *second) {
    if (!P) return fail(OZ_ERR_ARG, "heff_plan_variants: plan is NULL");
    if (first) *first = P->varL;
    if (second) *second = P->varR;
    return OZ_OK;
}

int heff_plan_launches(heff_plan P, int32_t *first, int32_t *second) {
    if (!P) return fail(OZ_ERR_ARG, "heff_plan_launches: plan is NULL");
    auto kind = [](const PairArgs &a) { return a.terms2 ? 3 : a.nwg > 0 ? 2 : a.stream_cus > 0 ? 1 : 0; };
    if (first) *first = P->S ? kind(P->chunks[0].argsL) : -1;
    if (second) *second = P->S ? kind(P->chunks[0].argsR) : -1;
    return OZ_OK;
}

int heff_plan_phase(heff_plan P, int phase, int32_t *variant, int32_t *order, int32_t *launch) {
    if (!P) return fail(OZ_ERR_ARG, "heff_plan_phase: plan is NULL");
    if (phase < 0 || phase > 1) return fail(OZ_ERR_ARG, "heff_plan_phase: phase = %d", phase);
    if (variant) *variant = P->choice[phase][0];
    if (order) *order = P->choice[phase][1];
    if (launch) *launch = P->choice[phase][2];
    return OZ_OK;
}

int heff_plan_chunks(heff_plan P) {
    if (!P) return fail(OZ_ERR_ARG, "heff_plan_chunks: plan is NULL");
    return static_cast<int>(P->chunks.size());
}

int64_t heff_plan_bytes(heff_plan P, int64_t *T_bytes) {
    if (!P) return fail(OZ_ERR_ARG, "heff_plan_bytes: plan is NULL");
    if (T_bytes) *T_bytes = static_cast<int64_t>(P->T_bytes);
    return static_cast<int64_t>(P->bytes);
}

double heff_flops(heff_plan P) { return P ? P->flops : 0.0; }

int heff_plan_destroy(heff_plan P) {
    if (!P) return OZ_OK;
    hipSetDevice(P->ctx->device);
    hipDeviceSynchronize();
    free_plan(P);
    return OZ_OK;
}

}  // extern "C"
