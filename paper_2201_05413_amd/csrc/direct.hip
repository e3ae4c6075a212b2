// direct.hip -- sparse Cholesky factorisation of A = K_II and its solves.
//
// The direct side of Sect. 4.3's multiple right-hand-side model: a direct
// solver factorises the matrix once (T_FACT) and then solves two triangular
// systems per right-hand side (T_SOLVE), one at a time or as a block
// (Eq. (3)).  A is symmetric positive definite, so the factorisation is
// Cholesky, A(perm, perm) = L L^T, computed by the multifrontal method:
//
//   ordering   geometric nested dissection on the DOF coordinates: a box is
//              split at the median coordinate of its longest side, and the
//              separator is the smaller of the two sets of DOFs that have a
//              matrix neighbour across the cut; both halves recurse, down to
//              leaves of at most kLeaf DOFs.  Positions follow the tree in
//              postorder (children before their separator).
//   symbolic   node k owns positions [b, e); its update set is every later
//              position coupled to its subtree: the later neighbours of its
//              own DOFs and the later entries of its children's update sets.
//              Its frontal matrix F (f = no + nu square, column-major) is
//              indexed by the own positions, then the update positions.
//   numeric    level by level from the deepest: F = A entries of the own
//              columns, plus the children's update matrices (extend-add, in
//              child order); partial Cholesky of the own columns:
//              L11 = chol(F11), L21 = F21 L11^-T, U = F22 - L21 L21^T.  The
//              panel [L11; L21] is kept; U goes to the parent.
//   solve      forward by levels from the deepest (y = L^-1 b, the update
//              vectors passed up by extend-add in child order), backward from
//              the root (x = L^-T y, reading the ancestors' x).
//
// Fronts up to kMidFront are factorised by one workgroup each (left-looking
// blocks of kFB columns, then the update block as one tiled product), their
// own blocks inverted in place, and solved by one workgroup per column
// chunk as matrix products.  Larger fronts whose own block has at most
// kMidFront columns go through level-wide kernels too: the own block by one
// workgroup, its inverse, then L21 = F21 L11^-T and U as tiled products.
// Only the fronts with larger own blocks call the libraries: rocSOLVER's
// POTRF and rocBLAS's TRSM / SYRK (dense FP64), then TRTRI for L11^-1.
// Every front thus keeps L11^-1 (and its transpose), so that the solves of
// the larger fronts are products spread over many workgroups instead of
// sequential substitutions.  Every sum has a fixed order, so the factor and
// the solution do not depend on the launch configuration or on the number
// of right-hand sides.
#include "engine.h"

#include <rocblas/rocblas.h>
#include <rocsolver/rocsolver.h>

#include <algorithm>
#include <array>
#include <atomic>
#include <cmath>
#include <numeric>
#include <thread>

namespace femcg {

constexpr int kLeaf = 64;         // nested-dissection leaves: at most this many DOFs
constexpr int kMidFront = 1024;   // fronts up to this size: one workgroup each
constexpr int kPanel = 8;         // columns per panel of the workgroup inversion of L11
constexpr int kInvLoads = 8;      // loads in flight per thread in that inversion's row products
constexpr int kFB = 16;           // columns per block column of the workgroup factorisation
constexpr int kFK = 256;          // finished columns per LDS stage of a block column's rows
constexpr int kRowsPT = 4;        // front rows per thread of the workgroup factorisation
constexpr int kSyT = 64;          // tile edge of the update-block product of the small fronts and of k_mid_l21
constexpr int kSyK = 32;          // columns of L21 per LDS stage of those
constexpr int kTriT = 128;        // tile edge of the update-block product of the larger fronts
constexpr int kTriK = 16;         // columns of L21 per LDS stage of that one
constexpr int kDBlock = 256;      // threads per workgroup of the direct kernels
constexpr int kSolveLds = 8192;   // doubles of LDS per solve workgroup (64 KB)
constexpr int kSolveLoads = 8;    // loads in flight per thread in the small fronts' solve products
constexpr int kWaveLanes = 64;    // lanes per wavefront
constexpr int kBigRows = 64;      // rows per workgroup of the larger fronts' row products (one per lane)
constexpr int kBigCols = 4;       // columns per workgroup of their column products
constexpr int kGatherRows = 256;  // rows of W per workgroup of the larger fronts' gathers
constexpr int kMirrorTile = 64;   // tile edge of the L11^-1 mirror

static_assert(kDBlock / kWaveLanes == 4, "the row products add four wave partials");
static_assert(kBigRows == kWaveLanes, "one row per lane");

// Larger fronts whose own block has at most kMidFront columns are factorised
// by the workgroup kernels rather than by per-front library calls (their
// update block's tiles must fit the grid's second dimension).
inline bool own_path(int64_t no, int64_t nu)
{
    const int64_t rt = (nu + kSyT - 1) / kSyT;
    return no > 0 && no <= kMidFront && rt * (rt + 1) / 2 <= 65535;
}

struct ChNode {
    int64_t b = 0, e = 0;          // own positions [b, e)
    int child[2] = {-1, -1};
    int parent = -1, depth = 0;
    std::vector<int64_t> upd;      // update positions, ascending, all >= e
    int64_t f() const { return (e - b) + (int64_t)upd.size(); }
    int64_t no() const { return e - b; }
    int64_t nu() const { return (int64_t)upd.size(); }
};

// Device-side description of one node.  Its frontal matrix (f x f, lower
// triangle) is stored in two parts: the panel columns 0..no-1 (f x no,
// ld f) in the panel store, where they become [L11; L21], and the update
// block U (rows and columns no..f-1; nu x nu, ld nu) in its level's buffer.
struct DNode {
    int64_t b;           // first own position
    int32_t no, nu;      // own and update sizes (f = no + nu)
    int64_t panel;       // offset of its panel in the panel store
    int64_t u;           // offset of its update block in its level's buffer
    int64_t wunit;       // solves: offset of its work block (f x t, ld f) in its level's buffer, in units of t
    int64_t idx;         // offset of its update positions in the index store (nu entries)
    int64_t rel[2];      // offsets of its children's relative indices in the index store
    int32_t child[2];    // node ids, -1 if none
};

}  // namespace femcg

struct fem_chol {
    int64_t n = 0;
    std::vector<int32_t> perm;                 // position -> free row
    std::vector<femcg::ChNode> nodes;
    std::vector<std::vector<int32_t>> levels;  // node ids by depth
    std::vector<femcg::DNode> hnodes;
    femcg::DNode *d_nodes = nullptr;
    int32_t *d_perm = nullptr;                 // position -> free row
    int64_t *d_index = nullptr;                // update positions and children's relative indices
    double *d_panel = nullptr;                 // panels [L11; L21] of every node, level by level
    char *d_lists = nullptr;                   // per-level work lists (one allocation)
    struct Level {
        int32_t *all = nullptr, *mid = nullptr;  // node ids: every node, fronts up to kMidFront
        int32_t nall = 0, nmid = 0;
        std::vector<int32_t> big;                // node ids of larger fronts (host loop)
        int32_t *dbig = nullptr;                 // the same on the device
        // larger fronts factorised by the workgroup kernels (own_path)
        int32_t *dbigtri = nullptr;
        int32_t nbigtri = 0;
        int32_t tri_rowtiles = 0, tri_tiles = 0;  // most F21 row tiles (k_mid_l21) and U tiles (k_mid_update)
        // solve items of the larger fronts, (node, first row or column) pairs:
        // columns of L11^-T (mirror), rows of L21, columns of L21, columns of L11^-1, rows of W (gathers)
        int32_t *prod[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
        int32_t nprod[5] = {0, 0, 0, 0, 0};
        int32_t mid_rows = 0;                    // largest f of the level's fronts up to kMidFront
        int32_t mid_tiles = 0;                   // most update-block tiles (k_mid_update) of those fronts
        int32_t solve_rows = 0;                  // LDS rows of the mid-front solves (largest f + no)
        int64_t panel0 = 0, panel1 = 0;          // the level's range in the panel store
        int64_t udoubles = 0;                    // update blocks of the level's nodes
        int64_t wunits = 0;                      // sum of f over the level's nodes
        int64_t *asm_dst = nullptr;              // A entries of the level's own columns
        double *asm_val = nullptr;
        int64_t nasm = 0;
        int32_t *ea_cols[2] = {nullptr, nullptr};  // (node, child column) pairs per child slot
        int64_t nea[2] = {0, 0};
    };
    std::vector<Level> lev;
    int64_t max_udoubles = 0, max_wunits = 0;
    int32_t *d_mir = nullptr;                  // mirror tiles of the larger fronts (node, tile code)
    int64_t nmir = 0;
    int32_t *d_fail = nullptr;                 // nonzero: a non-positive pivot
    chol_stats_t stats{};
    rocblas_handle blas = nullptr;
    ~fem_chol();
};

namespace femcg {
namespace {

// --------------------------------------------------------------------------
// host: ordering and symbolic analysis
// --------------------------------------------------------------------------

struct Graph {
    std::vector<int64_t> ptr;  // pruned pattern of A without the diagonal
    std::vector<int32_t> adj;
};

// The solver copy's pruning: entries |a| <= 4 eps max_row |a| are dropped
// (never the diagonal); they are zero in exact arithmetic (structural zeros
// of the element matrices).
static double prune_threshold(const HostSystem &hs, int64_t i)
{
    double mx = 0.0;
    for (int64_t t = hs.a_rowptr[i]; t < hs.a_rowptr[i + 1]; ++t) mx = std::max(mx, std::fabs(hs.a_val[t]));
    return 4.0 * 2.220446049250313e-16 * mx;
}

static void build_graph(const HostSystem &hs, Graph &G)
{
    const int64_t n = hs.nfree;
    G.ptr.assign(n + 1, 0);
    std::vector<int64_t> cnt(n, 0);
    parallel_for(n, [&](int64_t i0, int64_t i1) {
        for (int64_t i = i0; i < i1; ++i) {
            const double thr = prune_threshold(hs, i);
            int64_t c = 0;
            for (int64_t t = hs.a_rowptr[i]; t < hs.a_rowptr[i + 1]; ++t)
                c += hs.a_col[t] != i && std::fabs(hs.a_val[t]) > thr;
            cnt[i] = c;
        }
    });
    for (int64_t i = 0; i < n; ++i) G.ptr[i + 1] = G.ptr[i] + cnt[i];
    G.adj.resize(G.ptr[n]);
    parallel_for(n, [&](int64_t i0, int64_t i1) {
        for (int64_t i = i0; i < i1; ++i) {
            const double thr = prune_threshold(hs, i);
            int64_t o = G.ptr[i];
            for (int64_t t = hs.a_rowptr[i]; t < hs.a_rowptr[i + 1]; ++t)
                if (hs.a_col[t] != i && std::fabs(hs.a_val[t]) > thr) G.adj[o++] = hs.a_col[t];
        }
    });
}

// One dissection context: its own marks and nodes, positions written from
// `next` into the shared permutation (disjoint ranges per context).
struct NdState {
    const HostSystem *hs;
    const Graph *G;
    std::vector<int32_t> mark;  // stamps
    int32_t stamp = 0;
    int64_t next = 0;           // next free position
    std::vector<int32_t> *perm;
    std::vector<ChNode> nodes;
};

// Subtrees above this depth are dissected on threads of their own (the
// result is the serial one: nodes and positions in the same postorder).
constexpr int kNdThreadDepth = 3;

// Run fn(i) for i in [0, count) on up to 16 threads, items taken in turn.
static void par_items(int64_t count, const std::function<void(int64_t)> &fn)
{
    unsigned hw = std::thread::hardware_concurrency();
    const int nt = (int)std::min<int64_t>(count, std::min<unsigned>(hw ? hw : 1, 16));
    if (nt <= 1) {
        for (int64_t i = 0; i < count; ++i) fn(i);
        return;
    }
    std::atomic<int64_t> next{0};
    std::vector<std::thread> th;
    for (int t = 0; t < nt; ++t)
        th.emplace_back([&] {
            for (int64_t i = next++; i < count; i = next++) fn(i);
        });
    for (auto &x : th) x.join();
}

static double coord(const NdState &S, int32_t i, int r)
{
    const HostSystem &hs = *S.hs;
    return hs.dof_coords[hs.free2dof[i] * hs.dim + r];
}

static int new_node(NdState &S, const std::vector<int32_t> &own, int depth)
{
    ChNode nd;
    nd.b = S.next;
    for (int32_t i : own) (*S.perm)[S.next++] = i;
    nd.e = S.next;
    nd.depth = depth;
    S.nodes.push_back(std::move(nd));
    return (int)S.nodes.size() - 1;
}

// Nested dissection of the free rows `ids`; returns the node id.
static int dissect(NdState &S, std::vector<int32_t> &ids, int depth)
{
    if ((int64_t)ids.size() <= kLeaf) return new_node(S, ids, depth);
    const int dim = S.hs->dim;
    double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
    for (int32_t i : ids)
        for (int r = 0; r < dim; ++r) {
            lo[r] = std::min(lo[r], coord(S, i, r));
            hi[r] = std::max(hi[r], coord(S, i, r));
        }
    int ax = 0;
    for (int r = 1; r < dim; ++r)
        if (hi[r] - lo[r] > hi[ax] - lo[ax]) ax = r;
    // split at the median coordinate; ties on the median value go right
    std::vector<int32_t> ord(ids);
    const size_t mid = ord.size() / 2;
    std::nth_element(ord.begin(), ord.begin() + mid, ord.end(), [&](int32_t a, int32_t c) {
        const double ca = coord(S, a, ax), cc = coord(S, c, ax);
        return ca < cc || (ca == cc && a < c);
    });
    const double vm = coord(S, ord[mid], ax);
    std::vector<int32_t> L, R;
    for (int32_t i : ids) (coord(S, i, ax) < vm ? L : R).push_back(i);
    if (L.empty() || R.empty()) {
        // every coordinate equal along the axis: split by the order above
        L.assign(ord.begin(), ord.begin() + mid);
        R.assign(ord.begin() + mid, ord.end());
    }
    // the two boundary sets; the smaller one is the separator
    const Graph &G = *S.G;
    auto boundary = [&](const std::vector<int32_t> &side, const std::vector<int32_t> &other) {
        ++S.stamp;
        for (int32_t j : other) S.mark[j] = S.stamp;
        std::vector<int32_t> bnd;
        for (int32_t i : side)
            for (int64_t t = G.ptr[i]; t < G.ptr[i + 1]; ++t)
                if (S.mark[G.adj[t]] == S.stamp) {
                    bnd.push_back(i);
                    break;
                }
        return bnd;
    };
    std::vector<int32_t> BL = boundary(L, R), BR = boundary(R, L);
    const bool left = BL.size() <= BR.size();
    std::vector<int32_t> sep = left ? BL : BR;
    std::vector<int32_t> &cut = left ? L : R;
    ++S.stamp;
    for (int32_t i : sep) S.mark[i] = S.stamp;
    cut.erase(std::remove_if(cut.begin(), cut.end(), [&](int32_t i) { return S.mark[i] == S.stamp; }), cut.end());
    ids.clear();
    ids.shrink_to_fit();
    int c0 = -1, c1 = -1;
    if (depth < kNdThreadDepth && !L.empty() && !R.empty()) {
        // the left subtree on a thread of its own, into positions
        // [next, next + |L|), with its own marks; its nodes are then
        // appended before the right subtree's, as the serial order has them
        NdState SL;
        SL.hs = S.hs;
        SL.G = S.G;
        SL.mark.assign(S.mark.size(), 0);
        SL.perm = S.perm;
        SL.next = S.next;
        S.next += (int64_t)L.size();
        std::thread tl([&] { dissect(SL, L, depth + 1); });
        NdState SR;
        SR.hs = S.hs;
        SR.G = S.G;
        SR.perm = S.perm;
        SR.next = S.next;
        SR.mark.swap(S.mark);  // the right subtree reuses this context's marks
        SR.stamp = S.stamp;
        dissect(SR, R, depth + 1);
        tl.join();
        S.mark.swap(SR.mark);
        S.stamp = SR.stamp;
        S.next = SR.next;
        const int off = (int)S.nodes.size();
        auto append = [&](std::vector<ChNode> &v, int base) {
            for (ChNode &nd : v) {
                for (int &c : nd.child)
                    if (c >= 0) c += base;
                if (nd.parent >= 0) nd.parent += base;
                S.nodes.push_back(std::move(nd));
            }
        };
        append(SL.nodes, off);
        c0 = (int)S.nodes.size() - 1;
        append(SR.nodes, (int)S.nodes.size());
        c1 = (int)S.nodes.size() - 1;
    } else {
        c0 = L.empty() ? -1 : dissect(S, L, depth + 1);
        c1 = R.empty() ? -1 : dissect(S, R, depth + 1);
    }
    const int k = new_node(S, sep, depth);
    S.nodes[k].child[0] = c0;
    S.nodes[k].child[1] = c1;
    if (c0 >= 0) S.nodes[c0].parent = k;
    if (c1 >= 0) S.nodes[c1].parent = k;
    return k;
}

}  // namespace

// Ordering, tree, update sets and the statistics of the factorisation.
int chol_symbolic(const HostSystem &hs, fem_chol &C)
{
    const double t0 = now_s();
    Graph G;
    build_graph(hs, G);
    NdState S;
    S.hs = &hs;
    S.G = &G;
    S.mark.assign(hs.nfree, 0);
    std::vector<int32_t> perm(hs.nfree, 0);
    S.perm = &perm;
    std::vector<int32_t> all(hs.nfree);
    std::iota(all.begin(), all.end(), 0);
    if (hs.nfree > 0) dissect(S, all, 0);
    C.n = hs.nfree;
    C.perm = std::move(perm);
    C.nodes = std::move(S.nodes);
    const double t1 = now_s();
    std::vector<int32_t> ipos(C.n);
    for (int64_t p = 0; p < C.n; ++p) ipos[C.perm[p]] = (int32_t)p;
    // levels (a node's children are one level deeper)
    int maxd = 0;
    for (const ChNode &nd : C.nodes) maxd = std::max(maxd, nd.depth);
    C.levels.assign(maxd + 1, {});
    for (size_t k = 0; k < C.nodes.size(); ++k) C.levels[C.nodes[k].depth].push_back((int32_t)k);
    // update sets, deepest level first; the nodes of a level in parallel:
    // the later neighbours of the own rows and the children's update
    // positions, sorted and made unique
    for (int d = maxd; d >= 0; --d) {
        const std::vector<int32_t> &lv = C.levels[d];
        par_items((int64_t)lv.size(), [&](int64_t li) {
            ChNode &nd = C.nodes[lv[li]];
            std::vector<int64_t> u;
            for (int64_t p = nd.b; p < nd.e; ++p) {
                const int32_t i = C.perm[p];
                for (int64_t t = G.ptr[i]; t < G.ptr[i + 1]; ++t) {
                    const int64_t q = ipos[G.adj[t]];
                    if (q >= nd.e) u.push_back(q);
                }
            }
            for (int c : nd.child)
                if (c >= 0)
                    for (int64_t q : C.nodes[c].upd)
                        if (q >= nd.e) u.push_back(q);
            std::sort(u.begin(), u.end());
            u.erase(std::unique(u.begin(), u.end()), u.end());
            nd.upd = std::move(u);
        });
    }
    chol_stats_t &st = C.stats;
    st.n = C.n;
    st.nodes = (int32_t)C.nodes.size();
    st.levels = maxd + 1;
    double nnzl = 0, flops = 0, panel = 0, peak = 0;
    int64_t maxf = 0;
    std::vector<double> lev(maxd + 1, 0.0);
    for (const ChNode &nd : C.nodes) {
        const double no = (double)nd.no(), nu = (double)nd.nu(), f = no + nu;
        nnzl += no * (no + 1) / 2 + nu * no;
        flops += no * no * no / 3.0 + nu * no * no + nu * nu * no;
        panel += f * no;
        maxf = std::max<int64_t>(maxf, nd.f());
        lev[nd.depth] += f * f;
    }
    for (int d = 0; d < maxd; ++d) peak = std::max(peak, lev[d] + lev[d + 1]);
    if (maxd == 0) peak = lev[0];
    st.nnz_l = (int64_t)nnzl;
    st.flops = flops;
    st.max_front = (int32_t)maxf;
    st.factor_mb = (panel * 8.0) * 1e-6;
    st.work_mb = (peak * 8.0) * 1e-6;
    st.order_s = t1 - t0;
    st.symbolic_s = now_s() - t1;
    return FEMCG_OK;
}


// --------------------------------------------------------------------------
// device kernels
// --------------------------------------------------------------------------

namespace {

// Element (r, c), r >= c, of a frontal matrix stored as panel + update block.
struct Front {
    double *panel, *u;
    int no, nu, f;
    __device__ double &at(int r, int c) const
    {
        return c < no ? panel[r + (int64_t)c * f] : u[(r - no) + (int64_t)(c - no) * nu];
    }
};

__device__ inline Front front_of(const DNode &D, double *panel, double *ubuf)
{
    return Front{panel + D.panel, ubuf + D.u, D.no, D.nu, D.no + D.nu};
}

// A's entries of the level's own columns (every frontal position written by
// exactly one entry; the panels were zeroed before).
__global__ __launch_bounds__(kDBlock) void k_assemble(const int64_t *dst, const double *val, int64_t n, double *panel)
{
    for (int64_t e = (int64_t)blockIdx.x * kDBlock + threadIdx.x; e < n; e += (int64_t)gridDim.x * kDBlock)
        panel[dst[e]] = val[e];
}

// Extend-add of child slot s: block = one (node, child column b) pair; the
// child's update column b is added into the node's front at the child's
// relative indices (rows rel[a] >= rel[b], since rel increases).
__global__ __launch_bounds__(kDBlock) void k_extend_add(const DNode *nodes, const int32_t *pairs, int s,
                                                        const int64_t *index, double *panel, double *ubuf,
                                                        const double *uchild)
{
    const int k = pairs[2 * blockIdx.x], b = pairs[2 * blockIdx.x + 1];
    const DNode D = nodes[k];
    const DNode Cn = nodes[D.child[s]];
    const Front F = front_of(D, panel, ubuf);
    const int64_t *rel = index + D.rel[s];
    const double *U = uchild + Cn.u;
    const int nuc = Cn.nu;
    const int cb = (int)rel[b];
    for (int a = b + threadIdx.x; a < nuc; a += kDBlock) F.at((int)rel[a], cb) += U[a + (int64_t)b * nuc];
}

// Own columns of one front (f <= kMidFront) per workgroup, left-looking in
// blocks of kFB columns: each thread holds up to kRowsPT rows r >= J of the
// block column and subtracts sum_k L(r, k) L(J + q, k) over the finished
// columns k < J (the block's rows L(J.., k) staged in LDS in chunks of kFK);
// the block's diagonal part is then factorised in LDS and the rows below
// (L21 included) solve against it.  The update block U = F22 - L21 L21^T
// follows in k_mid_update.  With diag_only, only the own block F11
// (no <= kMidFront) is factorised, in place in the panel (ld f): the larger
// fronts' L21 and U then come from TRSM and SYRK.  Every sum runs over k in
// one fixed order.
__global__ __launch_bounds__(kDBlock) void k_mid_factor(const DNode *nodes, const int32_t *list, double *panel,
                                                        int32_t *fail, int diag_only)
{
    __shared__ double S[kFK * kFB];
    __shared__ double Dg[kFB][kFB + 1];
    __shared__ int s_bad;
    static_assert(kRowsPT * kDBlock >= kMidFront, "every row of a front has a thread");
    const DNode D = nodes[list[blockIdx.x]];
    const int ld = D.no + D.nu, no = D.no, tid = threadIdx.x;
    const int f = diag_only ? no : ld;  // rows processed
    double *A = panel + D.panel;
    if (tid == 0) s_bad = 0;
    for (int J = 0; J < no; J += kFB) {
        const int jw = min(kFB, no - J);
        double acc[kRowsPT][kFB];
#pragma unroll
        for (int i = 0; i < kRowsPT; ++i) {
            const int r = J + tid + i * kDBlock;
#pragma unroll
            for (int q = 0; q < kFB; ++q) acc[i][q] = (r < f && q < jw) ? A[r + (int64_t)(J + q) * ld] : 0.0;
        }
        for (int kc = 0; kc < J; kc += kFK) {
            const int kw = min(kFK, J - kc);
            __syncthreads();
            for (int e = tid; e < kw * kFB; e += kDBlock) {
                const int kk = e / kFB, q = e % kFB;
                S[e] = q < jw ? A[(J + q) + (int64_t)(kc + kk) * ld] : 0.0;
            }
            __syncthreads();
#pragma unroll 4
            for (int kk = 0; kk < kw; ++kk) {
                const double *sk = S + kk * kFB;
                double l[kRowsPT];
#pragma unroll
                for (int i = 0; i < kRowsPT; ++i) {
                    const int r = J + tid + i * kDBlock;
                    l[i] = r < f ? A[r + (int64_t)(kc + kk) * ld] : 0.0;
                }
#pragma unroll
                for (int q = 0; q < kFB; ++q) {
                    const double sq = sk[q];
#pragma unroll
                    for (int i = 0; i < kRowsPT; ++i) acc[i][q] -= l[i] * sq;
                }
            }
        }
        // the block's diagonal part: rows J..J+jw-1 are threads 0..jw-1, first row slot
        if (tid < jw)
#pragma unroll
            for (int q = 0; q < kFB; ++q) Dg[tid][q] = acc[0][q];
        __syncthreads();
        for (int j = 0; j < jw; ++j) {
            if (tid == 0) {
                const double d = Dg[j][j];
                if (!(d > 0.0)) s_bad = 1;
                Dg[j][j] = sqrt(d > 0.0 ? d : 1.0);
            }
            __syncthreads();
            if (tid > j && tid < jw) Dg[tid][j] /= Dg[j][j];
            __syncthreads();
            if (tid > j && tid < jw)
                for (int q = j + 1; q <= tid; ++q) Dg[tid][q] -= Dg[tid][j] * Dg[q][j];
            __syncthreads();
        }
        if (tid < jw)
            for (int q = 0; q <= tid; ++q) A[(J + tid) + (int64_t)(J + q) * ld] = Dg[tid][q];
        // the rows below: x L_JJ^T = acc, by forward substitution over q
#pragma unroll
        for (int i = 0; i < kRowsPT; ++i) {
            const int r = J + tid + i * kDBlock;
            if (r < J + jw || r >= f) continue;
            double x[kFB];
#pragma unroll
            for (int q = 0; q < kFB; ++q) {
                double v = acc[i][q];
#pragma unroll
                for (int p = 0; p < q; ++p) v -= x[p] * Dg[q][p];
                x[q] = q < jw ? v / Dg[q][q] : 0.0;
                if (q < jw) A[r + (int64_t)(J + q) * ld] = x[q];
            }
        }
        __syncthreads();
    }
    if (tid == 0 && s_bad) fail[0] = 1;
}

// U = F22 - L21 L21^T after the own columns: one workgroup per (front,
// TT x TT tile of U's lower triangle, blockIdx.y in row order).  L21 goes
// through LDS in chunks of KS columns; the next chunk is loaded into
// registers while the current one is summed.  Each thread sums a
// (TT / 16) x (TT / 16) block of the tile over k in order.
template <int TT, int KS>
__global__ __launch_bounds__(kDBlock) void k_mid_update(const DNode *nodes, const int32_t *list, const double *panel,
                                                        double *ubuf)
{
    constexpr int RT = TT / 16;                  // rows and columns per thread
    constexpr int NL = 2 * KS * TT / kDBlock;    // staged values per thread and chunk
    static_assert(NL * kDBlock == 2 * KS * TT && TT % 16 == 0, "whole chunks per thread");
    __shared__ double St[2 * KS * TT];           // [0]: L21 rows of the tile rows, [1]: of its columns; [kk][m]
    const DNode D = nodes[list[blockIdx.x]];
    const int no = D.no, nu = D.nu, ld = no + nu, tid = threadIdx.x;
    int ti = 0, tj = (int)blockIdx.y;
    while (tj > ti) tj -= ++ti;  // row ti holds tiles 0..ti
    if (no == 0 || ti * TT >= nu) return;  // the same for the whole workgroup
    const double *A = panel + D.panel;
    double *U = ubuf + D.u;
    const int tx = tid % 16, ty = tid / 16;
    const int R0 = ti * TT, C0 = tj * TT;
    double c[RT][RT], pf[NL];
#pragma unroll
    for (int i = 0; i < RT; ++i)
#pragma unroll
        for (int j = 0; j < RT; ++j) c[i][j] = 0.0;
    auto fetch = [&](int k0) {
#pragma unroll
        for (int v = 0; v < NL; ++v) {
            const int e = tid + v * kDBlock, h = e / (KS * TT), e2 = e % (KS * TT);
            const int k = k0 + e2 / TT, row = (h ? C0 : R0) + e2 % TT;
            pf[v] = (k < no && row < nu) ? A[(no + row) + (int64_t)k * ld] : 0.0;
        }
    };
    fetch(0);
    for (int k0 = 0; k0 < no; k0 += KS) {
        __syncthreads();
#pragma unroll
        for (int v = 0; v < NL; ++v) St[tid + v * kDBlock] = pf[v];
        __syncthreads();
        if (k0 + KS < no) fetch(k0 + KS);
        const int kw = min(KS, no - k0);
        for (int kk = 0; kk < kw; ++kk) {
            double av[RT], bv[RT];
#pragma unroll
            for (int i = 0; i < RT; ++i) av[i] = St[kk * TT + tx + 16 * i];
#pragma unroll
            for (int j = 0; j < RT; ++j) bv[j] = St[KS * TT + kk * TT + ty + 16 * j];
#pragma unroll
            for (int i = 0; i < RT; ++i)
#pragma unroll
                for (int j = 0; j < RT; ++j) c[i][j] += av[i] * bv[j];
        }
    }
#pragma unroll
    for (int i = 0; i < RT; ++i)
#pragma unroll
        for (int j = 0; j < RT; ++j) {
            const int ra = R0 + tx + 16 * i, cb = C0 + ty + 16 * j;
            if (ra < nu && cb <= ra) U[ra + (int64_t)cb * nu] -= c[i][j];
        }
}

// L21 = F21 L11^-T of the larger fronts whose own block has at most
// kMidFront columns, once k_mid_inv has left L11^-1 in the own block: one
// workgroup per (front, kSyT rows of F21, blockIdx.y), in place.  Column
// tiles of kSyT go from the last to the first: the entries of a tile's
// columns c are sum_{k <= c} F21(r, k) L11^-1(c, k), and only columns left
// of the tile are read after it is written.  L11^-1(c, k) is read from the
// lower triangle (k <= c) only.  Chunks of kSyK go through LDS, the next one
// loaded into registers while the current one is summed.
__global__ __launch_bounds__(kDBlock) void k_mid_l21(const DNode *nodes, const int32_t *list, double *panel)
{
    constexpr int NL = 2 * kSyK * kSyT / kDBlock;  // staged values per thread and chunk
    __shared__ double St[2 * kSyK * kSyT];          // [0]: F21(tile row m, k), [1]: L11^-1(tile column m, k); [kk][m]
    const DNode D = nodes[list[blockIdx.x]];
    const int no = D.no, nu = D.nu, ld = no + nu, tid = threadIdx.x;
    const int R0 = (int)blockIdx.y * kSyT;
    if (no == 0 || R0 >= nu) return;  // the same for the whole workgroup
    double *A = panel + D.panel;
    const int tx = tid % 16, ty = tid / 16;
    double pf[NL];
    auto fetch = [&](int C0, int k0, int kend) {
#pragma unroll
        for (int v = 0; v < NL; ++v) {
            const int e = tid + v * kDBlock, h = e / (kSyK * kSyT), e2 = e % (kSyK * kSyT);
            const int k = k0 + e2 / kSyT, m = e2 % kSyT;
            if (h == 0) pf[v] = (k < kend && R0 + m < nu) ? A[(no + R0 + m) + (int64_t)k * ld] : 0.0;
            else pf[v] = (k < kend && C0 + m < no && k <= C0 + m) ? A[(C0 + m) + (int64_t)k * ld] : 0.0;
        }
    };
    for (int C0 = ((no - 1) / kSyT) * kSyT; C0 >= 0; C0 -= kSyT) {
        const int kend = min(no, C0 + kSyT);
        double c[4][4];
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = 0; j < 4; ++j) c[i][j] = 0.0;
        fetch(C0, 0, kend);
        for (int k0 = 0; k0 < kend; k0 += kSyK) {
            __syncthreads();
#pragma unroll
            for (int v = 0; v < NL; ++v) St[tid + v * kDBlock] = pf[v];
            __syncthreads();
            if (k0 + kSyK < kend) fetch(C0, k0 + kSyK, kend);
            const int kw = min(kSyK, kend - k0);
            for (int kk = 0; kk < kw; ++kk) {
                double av[4], bv[4];
#pragma unroll
                for (int i = 0; i < 4; ++i) av[i] = St[kk * kSyT + tx + 16 * i];
#pragma unroll
                for (int j = 0; j < 4; ++j) bv[j] = St[kSyK * kSyT + kk * kSyT + ty + 16 * j];
#pragma unroll
                for (int i = 0; i < 4; ++i)
#pragma unroll
                    for (int j = 0; j < 4; ++j) c[i][j] += av[i] * bv[j];
            }
        }
        __syncthreads();  // every read of the tile's columns precedes its stores
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int ra = R0 + tx + 16 * i, cb = C0 + ty + 16 * j;
                if (ra < nu && cb < no) A[(no + ra) + (int64_t)cb * ld] = c[i][j];
            }
    }
}

// ---- solves: z holds the right-hand sides in elimination order, [n][t] ----

// z[p][c] = B[perm[p]][c]   /   X[perm[p]][c] = z[p][c]
__global__ __launch_bounds__(kDBlock) void k_permute(const int32_t *perm, int64_t n, int t, const double *src,
                                                     double *dst, int to_positions)
{
    const int64_t tot = n * t;
    for (int64_t e = (int64_t)blockIdx.x * kDBlock + threadIdx.x; e < tot; e += (int64_t)gridDim.x * kDBlock) {
        const int64_t p = e / t, c = e - p * t;
        const int64_t i = perm[p];
        if (to_positions) dst[e] = src[i * t + c];
        else dst[i * t + c] = src[e];
    }
}

// Forward gather of one node into its work block W (f x t, ld f), columns
// [c0, c0 + tc): its own right-hand-side rows, zeros below, then the
// children's update vectors (rows no_c..f_c of their blocks) added at their
// relative indices, child 0 first.  One workgroup; complete on return.
__device__ void fwd_gather(const DNode &D, const DNode *nodes, const int64_t *index, const double *z, int t,
                           double *W, const double *wchild, int c0, int tc)
{
    const int f = D.no + D.nu;
    for (int64_t e = threadIdx.x; e < (int64_t)f * tc; e += kDBlock) {
        const int c = c0 + (int)(e / f), r = (int)(e % f);
        W[r + (int64_t)c * f] = r < D.no ? z[(D.b + r) * t + c] : 0.0;
    }
    for (int s = 0; s < 2; ++s) {
        __syncthreads();
        if (D.child[s] < 0) continue;
        const DNode Cn = nodes[D.child[s]];
        const int fc = Cn.no + Cn.nu;
        const double *V = wchild + Cn.wunit * t;
        const int64_t *rel = index + D.rel[s];
        for (int64_t e = threadIdx.x; e < (int64_t)Cn.nu * tc; e += kDBlock) {
            const int c = c0 + (int)(e / Cn.nu), a = (int)(e % Cn.nu);
            W[rel[a] + (int64_t)c * f] += V[(Cn.no + a) + (int64_t)c * fc];
        }
    }
    __syncthreads();
}

// sum over k in [k0, k1) of P[k * ps] * S[k * ss], in order of k, with
// kSolveLoads loads of P in flight (the trip counts vary, so the compiler
// does not unroll these loops by itself)
__device__ __forceinline__ double strided_dot(const double *P, int64_t ps, const double *S, int ss, int k0, int k1)
{
    double acc = 0.0;
    int k = k0;
    for (; k + kSolveLoads <= k1; k += kSolveLoads) {
        double x[kSolveLoads];
#pragma unroll
        for (int u = 0; u < kSolveLoads; ++u) x[u] = P[(int64_t)(k + u) * ps];
#pragma unroll
        for (int u = 0; u < kSolveLoads; ++u) acc += x[u] * S[(k + u) * ss];
    }
    for (; k < k1; ++k) acc += P[(int64_t)k * ps] * S[k * ss];
    return acc;
}

// Solves of a front up to kMidFront, whose own block holds L11^-1 (lower
// triangle, diagonal included) and its transpose (strictly upper
// triangle), so that both triangular solves are products.  One workgroup
// per (front, chunk of cw right-hand-side columns, blockIdx.y); the chunk
// of W is staged in LDS as S (f x tc) with the product in T (no x tc).
// Threads take (row, column) pairs with the rows fastest, so that the
// factor's loads of a wave are contiguous; every sum runs over its index
// in one fixed order.  Dynamic LDS: kSolveLds doubles, (f + no) x cw fit.

// Forward: gather, y = L11^-1 w (rows of L11^-1), w_upd -= L21 y; y to z,
// w_upd back to W for the parent's gather.
__global__ __launch_bounds__(kDBlock) void k_mid_fwd(const DNode *nodes, const int32_t *list, const int64_t *index,
                                                     const double *panel, double *z, int t, int cw, double *wbuf,
                                                     const double *wchild)
{
    extern __shared__ double S[];
    const DNode D = nodes[list[blockIdx.x]];
    const int no = D.no, nu = D.nu, f = no + nu, tid = threadIdx.x;
    const int c0 = blockIdx.y * cw, tc = min(cw, t - c0);
    double *W = wbuf + D.wunit * t;
    const double *P = panel + D.panel;
    double *T = S + (int64_t)f * tc;
    fwd_gather(D, nodes, index, z, t, W, wchild, c0, tc);  // ends with a barrier
    for (int64_t e = tid; e < (int64_t)f * tc; e += kDBlock) {
        const int c = (int)(e / f), r = (int)(e % f);
        S[r * tc + c] = W[r + (int64_t)(c0 + c) * f];
    }
    __syncthreads();
    for (int64_t e = tid; e < (int64_t)no * tc; e += kDBlock) {
        const int c = (int)(e / no), i = (int)(e % no);
        T[i * tc + c] = strided_dot(P + i, f, S + c, tc, 0, i + 1);
    }
    __syncthreads();
    for (int64_t e = tid; e < (int64_t)nu * tc; e += kDBlock) {
        const int c = (int)(e / nu), r = no + (int)(e % nu);
        W[r + (int64_t)(c0 + c) * f] = S[r * tc + c] - strided_dot(P + r, f, T + c, tc, 0, no);
    }
    for (int64_t e = tid; e < (int64_t)no * tc; e += kDBlock) {
        const int c = (int)(e / no), i = (int)(e % no);
        z[(D.b + i) * t + c0 + c] = T[i * tc + c];
    }
}

// Backward: own rows (y) and update rows (the ancestors' x) from z,
// w = y - L21^T x_upd (columns of L21), x = L11^-T w (columns of the
// transpose in the upper triangle); x to z.
__global__ __launch_bounds__(kDBlock) void k_mid_bwd(const DNode *nodes, const int32_t *list, const int64_t *index,
                                                     const double *panel, double *z, int t, int cw)
{
    extern __shared__ double S[];
    const DNode D = nodes[list[blockIdx.x]];
    const int no = D.no, nu = D.nu, f = no + nu, tid = threadIdx.x;
    const int c0 = blockIdx.y * cw, tc = min(cw, t - c0);
    const double *P = panel + D.panel;
    const int64_t *upd = index + D.idx;
    double *T = S + (int64_t)f * tc;
    for (int64_t e = tid; e < (int64_t)f * tc; e += kDBlock) {
        const int c = (int)(e / f), r = (int)(e % f);
        S[r * tc + c] = r < no ? z[(D.b + r) * t + c0 + c] : z[upd[r - no] * t + c0 + c];
    }
    __syncthreads();
    for (int64_t e = tid; e < (int64_t)no * tc; e += kDBlock) {
        const int c = (int)(e / no), i = (int)(e % no);
        const double *Li = P + no + (int64_t)i * f;
        const double *Sa = S + (int64_t)no * tc + c;
        // four interleaved partial sums, combined in a fixed order
        double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
        int a = 0;
        for (; a + 4 <= nu; a += 4) {
            a0 += Li[a] * Sa[(int64_t)a * tc];
            a1 += Li[a + 1] * Sa[(int64_t)(a + 1) * tc];
            a2 += Li[a + 2] * Sa[(int64_t)(a + 2) * tc];
            a3 += Li[a + 3] * Sa[(int64_t)(a + 3) * tc];
        }
        for (; a < nu; ++a) a0 += Li[a] * Sa[(int64_t)a * tc];
        T[i * tc + c] = S[i * tc + c] - ((a0 + a1) + (a2 + a3));
    }
    __syncthreads();
    for (int64_t e = tid; e < (int64_t)no * tc; e += kDBlock) {
        const int c = (int)(e / no), j = (int)(e % no);
        z[(D.b + j) * t + c0 + c] = strided_dot(P + j, f, T + c, tc, j, no);
    }
}

// In-place inversion of the own block of fronts up to kMidFront (after the
// factorisation), one workgroup per front, then its transpose into the
// strictly upper triangle.  Panels of kPanel columns from the last: with
// the panel's diagonal block Dp, the rows below it L21p and the already
// inverted trailing block X22, the rows below become -X22 L21p Dp^-1 and the
// diagonal block Dp^-1.  Dynamic LDS: max(no * kPanel, transpose tile)
// doubles.
__global__ __launch_bounds__(kDBlock) void k_mid_inv(const DNode *nodes, const int32_t *list, double *panel)
{
    extern __shared__ double S[];
    __shared__ double Dm[kPanel][kPanel], Di[kPanel][kPanel];
    const DNode D = nodes[list[blockIdx.x]];
    const int no = D.no, f = no + D.nu, tid = threadIdx.x;
    double *P = panel + D.panel;
    for (int k0 = ((no - 1) / kPanel) * kPanel; k0 >= 0 && no > 0; k0 -= kPanel) {
        const int kw = min(kPanel, no - k0), r0 = k0 + kw, m = no - r0;
        for (int e = tid; e < kPanel * kPanel; e += kDBlock) {
            const int i = e / kPanel, j = e % kPanel;  // Dm[i][j] = L(k0 + i, k0 + j)
            Dm[i][j] = (i < kw && j <= i) ? P[(k0 + i) + (int64_t)(k0 + j) * f] : 0.0;
        }
        for (int e = tid; e < m * kw; e += kDBlock) {
            const int r = e / kw, c = e % kw;
            S[r * kPanel + c] = P[(r0 + r) + (int64_t)(k0 + c) * f];
        }
        __syncthreads();
        if (tid < kw) {  // column c of Dp^-1 by forward substitution
            const int c = tid;
            double x[kPanel];
#pragma unroll
            for (int i = 0; i < kPanel; ++i) {
                double v = i == c ? 1.0 : 0.0;
#pragma unroll
                for (int j = 0; j < i; ++j) v -= Dm[i][j] * x[j];
                x[i] = (i < kw && i >= c) ? v / Dm[i][i] : 0.0;
            }
#pragma unroll
            for (int i = 0; i < kPanel; ++i) Di[i][c] = x[i];
        }
        __syncthreads();
        for (int r = tid; r < m; r += kDBlock) {
            const int gi = r0 + r;
            double acc[kPanel];
#pragma unroll
            for (int c = 0; c < kPanel; ++c) acc[c] = 0.0;
            // X22's row in groups of kInvLoads loads, summed in order of j
            int j = r0;
            for (; j + kInvLoads <= gi + 1; j += kInvLoads) {
                double x[kInvLoads];
#pragma unroll
                for (int u = 0; u < kInvLoads; ++u) x[u] = P[gi + (int64_t)(j + u) * f];
#pragma unroll
                for (int u = 0; u < kInvLoads; ++u)
#pragma unroll
                    for (int c = 0; c < kPanel; ++c) acc[c] += x[u] * S[(j + u - r0) * kPanel + c];
            }
            for (; j <= gi; ++j) {
                const double x = P[gi + (int64_t)j * f];
#pragma unroll
                for (int c = 0; c < kPanel; ++c) acc[c] += x * S[(j - r0) * kPanel + c];
            }
            for (int c = 0; c < kw; ++c) {
                double v = 0.0;
                for (int q = c; q < kw; ++q) v += acc[q] * Di[q][c];
                P[gi + (int64_t)(k0 + c) * f] = -v;
            }
        }
        for (int e = tid; e < kw * kw; e += kDBlock) {
            const int i = e / kw, c = e % kw;
            if (i >= c) P[(k0 + i) + (int64_t)(k0 + c) * f] = Di[i][c];
        }
        __syncthreads();
    }
    // the transpose into the strictly upper triangle, one tile at a time
    constexpr int TT = kMirrorTile / 2;
    const int nt = (no + TT - 1) / TT;
    for (int ti = 0; ti < nt; ++ti)
        for (int tj = 0; tj <= ti; ++tj) {
            const int ro = ti * TT, co = tj * TT;
            for (int e = tid; e < TT * TT; e += kDBlock) {
                const int c = e / TT, r = e % TT;
                const int gr = ro + r, gc = co + c;
                S[c * (TT + 1) + r] = (gr < no && gr > gc) ? P[gr + (int64_t)gc * f] : 0.0;
            }
            __syncthreads();
            for (int e = tid; e < TT * TT; e += kDBlock) {
                const int r = e / TT, c = e % TT;
                const int gr = ro + r, gc = co + c;
                if (gr < no && gr > gc) P[gc + (int64_t)gr * f] = S[c * (TT + 1) + r];
            }
            __syncthreads();
        }
}

// Gathers of the larger fronts, one workgroup per (node, chunk of
// kGatherRows rows of W), every column.  Forward: own right-hand-side rows
// or zeros, then the children's update rows that land in the chunk (the
// relative indices increase, so they form one range), child 0 first.
__device__ inline int lower_index(const int64_t *rel, int n, int64_t v)
{
    int lo = 0, hi = n;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (rel[mid] < v) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

__global__ __launch_bounds__(kDBlock) void k_big_fwd_gather(const DNode *nodes, const int32_t *items,
                                                            const int64_t *index, const double *z, int t,
                                                            double *wbuf, const double *wchild)
{
    const DNode D = nodes[items[2 * blockIdx.x]];
    const int f = D.no + D.nu;
    const int r0 = items[2 * blockIdx.x + 1], r1 = min(f, r0 + kGatherRows), nr = r1 - r0;
    double *W = wbuf + D.wunit * t;
    for (int64_t e = threadIdx.x; e < (int64_t)nr * t; e += kDBlock) {
        const int c = (int)(e / nr), r = r0 + (int)(e % nr);
        W[r + (int64_t)c * f] = r < D.no ? z[(D.b + r) * t + c] : 0.0;
    }
    for (int s = 0; s < 2; ++s) {
        __syncthreads();
        if (D.child[s] < 0) continue;
        const DNode Cn = nodes[D.child[s]];
        const int fc = Cn.no + Cn.nu;
        const double *V = wchild + Cn.wunit * t;
        const int64_t *rel = index + D.rel[s];
        const int a0 = lower_index(rel, Cn.nu, r0), na = lower_index(rel, Cn.nu, r1) - a0;
        for (int64_t e = threadIdx.x; e < (int64_t)na * t; e += kDBlock) {
            const int c = (int)(e / na), a = a0 + (int)(e % na);
            W[rel[a] + (int64_t)c * f] += V[(Cn.no + a) + (int64_t)c * fc];
        }
    }
}

__global__ __launch_bounds__(kDBlock) void k_big_bwd_gather(const DNode *nodes, const int32_t *items,
                                                            const int64_t *index, const double *z, int t,
                                                            double *wbuf)
{
    const DNode D = nodes[items[2 * blockIdx.x]];
    const int f = D.no + D.nu;
    const int r0 = items[2 * blockIdx.x + 1], r1 = min(f, r0 + kGatherRows), nr = r1 - r0;
    const int64_t *upd = index + D.idx;
    double *W = wbuf + D.wunit * t;
    for (int64_t e = threadIdx.x; e < (int64_t)nr * t; e += kDBlock) {
        const int c = (int)(e / nr), r = r0 + (int)(e % nr);
        W[r + (int64_t)c * f] = r < D.no ? z[(D.b + r) * t + c] : z[upd[r - D.no] * t + c];
    }
}

// ---- larger fronts: solves in product form ----
// A front above kMidFront keeps L11^-1 (lower triangle, from TRTRI after
// its factorisation) in place of L11, so that both of its triangular solves
// are matrix products with no sequential dependence:
//   forward   y = L11^-1 w_own (to z),   w_upd -= L21 y
//   backward  w_own -= L21^T x_upd,      x = L11^-T w_own (to z)
// Right-hand-side columns come in chunks of TC (blockIdx.y); every column's
// sums run in the same order whatever t is.

// Row products: one workgroup per (node, chunk of 64 rows of L21), one row
// per lane; the four waves take contiguous quarters of the columns and their
// partial sums are added in wave order.  Rows of L21 times y (z's own
// rows), subtracted from W's update rows.
template <int TC>
__global__ __launch_bounds__(kDBlock) void k_big_rows(const DNode *nodes, const int32_t *items, const double *panel,
                                                      const double *z, int t, double *wbuf)
{
    __shared__ double part[kDBlock / kWaveLanes][TC][kWaveLanes];
    const DNode D = nodes[items[2 * blockIdx.x]];
    const int r0 = items[2 * blockIdx.x + 1];
    const int f = D.no + D.nu;
    const int c0 = blockIdx.y * TC, tcn = min(TC, t - c0);
    const int lane = threadIdx.x & (kWaveLanes - 1);
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWaveLanes);
    const int r = r0 + lane;
    const bool ok = r < D.nu;
    const int64_t prow = D.no + (ok ? r : D.nu - 1);
    const int per = (D.no + 3) / 4;
    const int js = min(D.no, wave * per), je = min(D.no, js + per);
    const double *P = panel + D.panel;
    double *W = wbuf + D.wunit * t;
    double acc[TC];
#pragma unroll
    for (int c = 0; c < TC; ++c) acc[c] = 0.0;
    // branch-free body (columns past tcn repeat the last one and are not
    // stored), so that the unrolled loads are all in flight together
#pragma unroll 16
    for (int j = js; j < je; ++j) {
        const double a = P[prow + (int64_t)j * f];
        const double *zj = z + (D.b + j) * t + c0;
#pragma unroll
        for (int c = 0; c < TC; ++c) acc[c] += a * zj[min(c, tcn - 1)];
    }
#pragma unroll
    for (int c = 0; c < TC; ++c) part[wave][c][lane] = acc[c];
    __syncthreads();
    if (threadIdx.x < kWaveLanes && ok)
        for (int c = 0; c < tcn; ++c) {
            const double v = (part[0][c][lane] + part[1][c][lane]) + (part[2][c][lane] + part[3][c][lane]);
            W[D.no + r + (int64_t)(c0 + c) * f] -= v;
        }
}

// Column products: one workgroup per (node, kBigCols consecutive columns);
// the four waves take contiguous quarters of the rows, each lane strides its
// quarter and reads every right-hand-side row once for all the workgroup's
// columns; lanes are added by a fixed xor tree, then the waves in order.
//   kL21   columns j of L21 against W's update rows, subtracted from W's own rows j
//   kLow   columns j of L11^-1 (rows j..no-1) against W's own rows: x_j, to z
//   kUp    columns j of L11^-T (rows 0..j, the mirror in the upper triangle)
//          against W's own rows: y_j = (L11^-1 w)_j, to z
enum ColForm { kL21 = 0, kLow = 1, kUp = 2 };
template <int TC>
__global__ __launch_bounds__(kDBlock) void k_big_cols(const DNode *nodes, const int32_t *items, int form,
                                                      const double *panel, double *z, int t, double *wbuf)
{
    __shared__ double part[kDBlock / kWaveLanes][kBigCols][TC];
    const DNode D = nodes[items[2 * blockIdx.x]];
    const int j0 = items[2 * blockIdx.x + 1], ncol = min(kBigCols, D.no - j0);
    const int lane = threadIdx.x & (kWaveLanes - 1);
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWaveLanes);
    const int f = D.no + D.nu;
    const int c0 = blockIdx.y * TC, tcn = min(TC, t - c0);
    // the rows any of the columns reads, split in four
    const int rs = form == kL21 ? D.no : (form == kLow ? j0 : 0);
    const int re = form == kL21 ? f : (form == kLow ? D.no : j0 + ncol);
    const int per = (re - rs + 3) / 4;
    const int ws = min(re, rs + wave * per), we = min(re, ws + per);
    const double *P = panel + D.panel + (int64_t)j0 * f;
    double *W = wbuf + D.wunit * t;
    double acc[kBigCols][TC];
#pragma unroll
    for (int q = 0; q < kBigCols; ++q)
#pragma unroll
        for (int c = 0; c < TC; ++c) acc[q][c] = 0.0;
    // branch-free body (columns past ncol and tcn repeat the last ones and
    // are not stored), so that the unrolled loads are all in flight together
#pragma unroll 4
    for (int r = ws + lane; r < we; r += kWaveLanes) {
        double wv[TC];
#pragma unroll
        for (int c = 0; c < TC; ++c) wv[c] = W[r + (int64_t)(c0 + min(c, tcn - 1)) * f];
#pragma unroll
        for (int q = 0; q < kBigCols; ++q) {
            // a 0/1 factor rather than a select, which the compiler turns
            // into a branch around the load (the factor's entries are finite)
            const bool skip = q >= ncol || (form == kLow && r < j0 + q) || (form == kUp && r > j0 + q);
            const double a = P[r + (int64_t)min(q, ncol - 1) * f] * (skip ? 0.0 : 1.0);
#pragma unroll
            for (int c = 0; c < TC; ++c) acc[q][c] += a * wv[c];
        }
    }
#pragma unroll
    for (int q = 0; q < kBigCols; ++q)
#pragma unroll
        for (int c = 0; c < TC; ++c) {
            double v = acc[q][c];
            for (int off = kWaveLanes / 2; off >= 1; off >>= 1) v += __shfl_xor(v, off, kWaveLanes);
            if (lane == 0) part[wave][q][c] = v;
        }
    __syncthreads();
    for (int e = threadIdx.x; e < ncol * tcn; e += kDBlock) {
        const int q = e / tcn, c = e % tcn, j = j0 + q;
        const double v = (part[0][q][c] + part[1][q][c]) + (part[2][q][c] + part[3][q][c]);
        if (form == kL21) W[j + (int64_t)(c0 + c) * f] -= v;
        else z[(D.b + j) * t + c0 + c] = v;
    }
}

// After TRTRI: the strictly lower triangle of L11^-1 copied, transposed,
// into the strictly upper triangle of the own block, one 64 x 64 tile per
// workgroup (items: node, tile row << 16 | tile column, tile row >= tile
// column), so that the forward product reads contiguous columns.
__global__ __launch_bounds__(kDBlock) void k_mirror(const DNode *nodes, const int32_t *items, double *panel)
{
    __shared__ double T[kMirrorTile][kMirrorTile + 1];
    const DNode D = nodes[items[2 * blockIdx.x]];
    const int code = items[2 * blockIdx.x + 1];
    const int r0 = (code >> 16) * kMirrorTile, c0 = (code & 0xffff) * kMirrorTile;
    const int f = D.no + D.nu;
    double *P = panel + D.panel;
    for (int e = threadIdx.x; e < kMirrorTile * kMirrorTile; e += kDBlock) {
        const int c = e / kMirrorTile, r = e % kMirrorTile;  // rows fastest: contiguous loads
        const int gr = r0 + r, gc = c0 + c;
        T[c][r] = (gr < D.no && gr > gc) ? P[gr + (int64_t)gc * f] : 0.0;
    }
    __syncthreads();
    for (int e = threadIdx.x; e < kMirrorTile * kMirrorTile; e += kDBlock) {
        const int r = e / kMirrorTile, c = e % kMirrorTile;  // target rows fastest: contiguous stores
        const int gr = r0 + r, gc = c0 + c;
        if (gr < D.no && gr > gc) P[gc + (int64_t)gr * f] = T[c][r];
    }
}

}  // namespace

// --------------------------------------------------------------------------
// host: numeric set-up, factorisation and solves
// --------------------------------------------------------------------------

#define DCHK(call)                                                                          \
    do {                                                                                    \
        hipError_t e_ = (call);                                                             \
        if (e_ != hipSuccess) return fail(FEMCG_EDEVICE, "%s: %s", #call, hipGetErrorString(e_)); \
    } while (0)
#define BCHK(call)                                                                          \
    do {                                                                                    \
        rocblas_status b_ = (call);                                                         \
        if (b_ != rocblas_status_success) return fail(FEMCG_EDEVICE, "%s: rocBLAS status %d", #call, (int)b_); \
    } while (0)

static int dgrid(int64_t work)
{
    return (int)std::max<int64_t>(1, std::min<int64_t>((work + kDBlock - 1) / kDBlock, 8192));
}

// Index of position q in node nd's front (own positions, then the update
// positions), or -1 if q is not in it (which the nested-dissection
// separators rule out; checked so that no kernel can index past a front).
static int64_t front_index(const ChNode &nd, int64_t q)
{
    if (q >= nd.b && q < nd.e) return q - nd.b;
    auto it = std::lower_bound(nd.upd.begin(), nd.upd.end(), q);
    if (it == nd.upd.end() || *it != q) return -1;
    return nd.no() + (it - nd.upd.begin());
}

// Offsets, index store, per-level lists and the assembly map; uploads them.
int chol_setup(const HostSystem &hs, fem_chol &C)
{
    const int64_t n = C.n;
    const size_t nn = C.nodes.size();
    std::vector<int32_t> ipos(n);
    for (int64_t p = 0; p < n; ++p) ipos[C.perm[p]] = (int32_t)p;
    C.hnodes.assign(nn, DNode{});
    const int nlev = (int)C.levels.size();
    C.lev.assign(nlev, fem_chol::Level{});
    int64_t panel = 0, nindex = 0;
    // offsets, deepest level first: panels in factorisation order; in the
    // index store each node's update positions, then its children's
    // relative indices
    for (int d = nlev - 1; d >= 0; --d) {
        fem_chol::Level &L = C.lev[d];
        L.panel0 = panel;
        int64_t u = 0, w = 0;
        for (int32_t k : C.levels[d]) {
            const ChNode &nd = C.nodes[k];
            DNode &D = C.hnodes[k];
            D.b = nd.b;
            D.no = (int32_t)nd.no();
            D.nu = (int32_t)nd.nu();
            D.panel = panel;
            panel += nd.f() * nd.no();
            D.u = u;
            u += nd.nu() * nd.nu();
            D.wunit = w;
            w += nd.f();
            D.idx = nindex;
            nindex += nd.nu();
            for (int s = 0; s < 2; ++s) {
                D.child[s] = nd.child[s];
                D.rel[s] = 0;
                if (nd.child[s] < 0) continue;
                D.rel[s] = nindex;
                nindex += C.nodes[nd.child[s]].nu();
            }
        }
        L.panel1 = panel;
        L.udoubles = u;
        L.wunits = w;
        C.max_udoubles = std::max(C.max_udoubles, u);
        C.max_wunits = std::max(C.max_wunits, w);
    }
    // the index store, nodes in parallel (binary searches in the fronts)
    std::vector<int64_t> index(nindex);
    std::atomic<int64_t> bad_upd{-1};
    par_items((int64_t)nn, [&](int64_t k) {
        const ChNode &nd = C.nodes[k];
        const DNode &D = C.hnodes[k];
        std::copy(nd.upd.begin(), nd.upd.end(), index.begin() + D.idx);
        for (int s = 0; s < 2; ++s) {
            if (nd.child[s] < 0) continue;
            int64_t o = D.rel[s];
            for (int64_t q : C.nodes[nd.child[s]].upd) {
                const int64_t r = front_index(nd, q);
                if (r < 0) bad_upd = q;
                index[o++] = r;
            }
        }
    });
    if (bad_upd >= 0)
        return fail(FEMCG_EINVAL, "chol: update position %lld outside the parent front", (long long)bad_upd.load());
    // assembly map: A entries (q >= p) of every own column p, level by
    // level in node order.  Nodes in parallel: a count, the offsets of the
    // nodes in their level's arrays, then each node writes its own range.
    std::vector<int32_t> lev_of(nn);
    for (int d = 0; d < nlev; ++d)
        for (int32_t k : C.levels[d]) lev_of[k] = d;
    auto kept = [&](int64_t p, int64_t i, int64_t t, double thr) {
        const int64_t j = hs.a_col[t];
        return !(ipos[j] < p || (j != i && !(std::fabs(hs.a_val[t]) > thr)));
    };
    std::vector<int64_t> acount(nn, 0), aoff(nn, 0);
    par_items((int64_t)nn, [&](int64_t k) {
        const ChNode &nd = C.nodes[k];
        int64_t c = 0;
        for (int64_t p = nd.b; p < nd.e; ++p) {
            const int64_t i = C.perm[p];
            const double thr = prune_threshold(hs, i);
            for (int64_t t = hs.a_rowptr[i]; t < hs.a_rowptr[i + 1]; ++t) c += kept(p, i, t, thr);
        }
        acount[k] = c;
    });
    std::vector<std::vector<int64_t>> adst(nlev);
    std::vector<std::vector<double>> aval(nlev);
    for (int d = 0; d < nlev; ++d) {
        int64_t tot = 0;
        for (int32_t k : C.levels[d]) {
            aoff[k] = tot;
            tot += acount[k];
        }
        adst[d].resize(tot);
        aval[d].resize(tot);
    }
    std::atomic<int64_t> bad_p{-1};
    par_items((int64_t)nn, [&](int64_t k) {
        const ChNode &nd = C.nodes[k];
        const DNode &D = C.hnodes[k];
        const int64_t f = nd.f();
        int64_t *dst = adst[lev_of[k]].data() + aoff[k];
        double *val = aval[lev_of[k]].data() + aoff[k];
        for (int64_t p = nd.b; p < nd.e; ++p) {
            const int64_t i = C.perm[p];
            const double thr = prune_threshold(hs, i);
            for (int64_t t = hs.a_rowptr[i]; t < hs.a_rowptr[i + 1]; ++t) {
                if (!kept(p, i, t, thr)) continue;
                const int64_t r = front_index(nd, ipos[hs.a_col[t]]);
                if (r < 0) bad_p = p;  // the call fails below
                *dst++ = D.panel + r + (p - nd.b) * f;
                *val++ = hs.a_val[t];
            }
        }
    });
    if (bad_p >= 0) return fail(FEMCG_EINVAL, "chol: a matrix entry of row %lld lies outside its front", (long long)bad_p.load());
    // device lists: per level node ids (all, mid, big), extend-add pairs, assembly
    size_t bytes = 0;
    auto reserve = [&](size_t b) {
        const size_t off = (bytes + 255) & ~(size_t)255;
        bytes = off + b;
        return off;
    };
    struct Off {
        size_t all, mid, big, bigtri, ea[2], dst, val, prod[5];
    };
    std::vector<Off> off(nlev);
    std::vector<std::vector<int32_t>> mid(nlev), big(nlev), bigtri(nlev), ea0(nlev), ea1(nlev);
    std::vector<std::array<std::vector<int32_t>, 5>> prod(nlev);
    std::vector<int32_t> mir;  // mirror tiles of every larger front
    std::vector<int64_t> eoff[2] = {std::vector<int64_t>(nn, 0), std::vector<int64_t>(nn, 0)};  // first pair of a node
    std::vector<int64_t> esz[2] = {std::vector<int64_t>(nlev, 0), std::vector<int64_t>(nlev, 0)};  // pairs per level
    for (int d = 0; d < nlev; ++d) {
        for (int32_t k : C.levels[d]) {
            const ChNode &nd = C.nodes[k];
            if (nd.f() <= kMidFront) {
                mid[d].push_back(k);
                C.lev[d].mid_rows = std::max<int32_t>(C.lev[d].mid_rows, (int32_t)nd.f());
                if (nd.no() > 0) {
                    const int32_t nt = (int32_t)((nd.nu() + kSyT - 1) / kSyT);
                    C.lev[d].mid_tiles = std::max<int32_t>(C.lev[d].mid_tiles, nt * (nt + 1) / 2);
                }
                C.lev[d].solve_rows = std::max<int32_t>(C.lev[d].solve_rows, (int32_t)(nd.f() + nd.no()));
            } else {
                big[d].push_back(k);
                if (own_path(nd.no(), nd.nu())) {
                    bigtri[d].push_back(k);
                    const int32_t rt = (int32_t)((nd.nu() + kSyT - 1) / kSyT);
                    const int32_t ut = (int32_t)((nd.nu() + kTriT - 1) / kTriT);
                    C.lev[d].tri_rowtiles = std::max(C.lev[d].tri_rowtiles, rt);
                    C.lev[d].tri_tiles = std::max(C.lev[d].tri_tiles, ut * (ut + 1) / 2);
                } else {
                    const int32_t nt = (int32_t)((nd.no() + kMirrorTile - 1) / kMirrorTile);
                    if (nt >= (1 << 15))
                        return fail(FEMCG_EINVAL, "chol: separator of %lld DOFs is too large", (long long)nd.no());
                    for (int32_t ti = 0; ti < nt; ++ti)
                        for (int32_t tj = 0; tj <= ti; ++tj) mir.insert(mir.end(), {k, (ti << 16) | tj});
                }
                auto &pr = prod[d];
                for (int32_t j = 0; j < (int32_t)nd.no(); j += kBigCols) pr[0].insert(pr[0].end(), {k, j});
                if (nd.no() > 0)
                    for (int32_t r = 0; r < (int32_t)nd.nu(); r += kBigRows) pr[1].insert(pr[1].end(), {k, r});
                if (nd.nu() > 0)
                    for (int32_t j = 0; j < (int32_t)nd.no(); j += kBigCols) pr[2].insert(pr[2].end(), {k, j});
                for (int32_t j = 0; j < (int32_t)nd.no(); j += kBigCols) pr[3].insert(pr[3].end(), {k, j});
                for (int32_t r = 0; r < (int32_t)nd.f(); r += kGatherRows) pr[4].insert(pr[4].end(), {k, r});
            }
            for (int s = 0; s < 2; ++s) {  // extend-add pairs: counted here, written below
                const int c = C.nodes[k].child[s];
                if (c < 0) continue;
                eoff[s][k] = esz[s][d];
                esz[s][d] += C.nodes[c].nu();
            }
        }
        off[d].all = reserve(C.levels[d].size() * 4);
        off[d].mid = reserve(mid[d].size() * 4);
        off[d].big = reserve(big[d].size() * 4);
        off[d].bigtri = reserve(bigtri[d].size() * 4);
        off[d].ea[0] = reserve(esz[0][d] * 8);
        off[d].ea[1] = reserve(esz[1][d] * 8);
        off[d].dst = reserve(adst[d].size() * 8);
        off[d].val = reserve(aval[d].size() * 8);
        for (int q = 0; q < 5; ++q) off[d].prod[q] = reserve(prod[d][q].size() * 4);
    }
    const size_t off_mir = reserve(mir.size() * 4);
    // the extend-add pairs (node, child column b), nodes in parallel, in the
    // order of the level's nodes
    for (int d = 0; d < nlev; ++d) {
        ea0[d].resize(2 * esz[0][d]);
        ea1[d].resize(2 * esz[1][d]);
    }
    par_items((int64_t)nn, [&](int64_t k) {
        for (int s = 0; s < 2; ++s) {
            const int c = C.nodes[k].child[s];
            if (c < 0) continue;
            int32_t *v = (s == 0 ? ea0 : ea1)[lev_of[k]].data() + 2 * eoff[s][k];
            for (int64_t b = 0; b < C.nodes[c].nu(); ++b) {
                v[2 * b] = (int32_t)k;
                v[2 * b + 1] = (int32_t)b;
            }
        }
    });
    DCHK(hipMalloc((void **)&C.d_lists, std::max<size_t>(bytes, 256)));
    DCHK(hipMalloc((void **)&C.d_nodes, sizeof(DNode) * std::max<size_t>(nn, 1)));
    DCHK(hipMalloc((void **)&C.d_perm, sizeof(int32_t) * std::max<int64_t>(n, 1)));
    DCHK(hipMalloc((void **)&C.d_index, sizeof(int64_t) * std::max<size_t>(index.size(), 1)));
    DCHK(hipMalloc((void **)&C.d_fail, sizeof(int32_t)));
    DCHK(hipMemcpy(C.d_nodes, C.hnodes.data(), sizeof(DNode) * nn, hipMemcpyHostToDevice));
    DCHK(hipMemcpy(C.d_perm, C.perm.data(), sizeof(int32_t) * n, hipMemcpyHostToDevice));
    if (!index.empty()) DCHK(hipMemcpy(C.d_index, index.data(), sizeof(int64_t) * index.size(), hipMemcpyHostToDevice));
    auto put = [&](size_t o, const void *src, size_t b) -> int {
        if (b) DCHK(hipMemcpy(C.d_lists + o, src, b, hipMemcpyHostToDevice));
        return FEMCG_OK;
    };
    {
        const int rc = put(off_mir, mir.data(), mir.size() * 4);
        if (rc) return rc;
        C.d_mir = (int32_t *)(C.d_lists + off_mir);
        C.nmir = (int64_t)mir.size() / 2;
    }
    for (int d = 0; d < nlev; ++d) {
        fem_chol::Level &L = C.lev[d];
        int rc;
        if ((rc = put(off[d].all, C.levels[d].data(), C.levels[d].size() * 4)) ||
            (rc = put(off[d].mid, mid[d].data(), mid[d].size() * 4)) ||
            (rc = put(off[d].big, big[d].data(), big[d].size() * 4)) ||
            (rc = put(off[d].bigtri, bigtri[d].data(), bigtri[d].size() * 4)) ||
            (rc = put(off[d].ea[0], ea0[d].data(), ea0[d].size() * 4)) ||
            (rc = put(off[d].ea[1], ea1[d].data(), ea1[d].size() * 4)) ||
            (rc = put(off[d].dst, adst[d].data(), adst[d].size() * 8)) ||
            (rc = put(off[d].val, aval[d].data(), aval[d].size() * 8)))
            return rc;
        for (int q = 0; q < 5; ++q) {
            if ((rc = put(off[d].prod[q], prod[d][q].data(), prod[d][q].size() * 4))) return rc;
            L.prod[q] = (int32_t *)(C.d_lists + off[d].prod[q]);
            L.nprod[q] = (int32_t)(prod[d][q].size() / 2);
        }
        L.all = (int32_t *)(C.d_lists + off[d].all);
        L.mid = (int32_t *)(C.d_lists + off[d].mid);
        L.nall = (int32_t)C.levels[d].size();
        L.nmid = (int32_t)mid[d].size();
        L.big = big[d];
        L.dbig = (int32_t *)(C.d_lists + off[d].big);
        L.dbigtri = (int32_t *)(C.d_lists + off[d].bigtri);
        L.nbigtri = (int32_t)bigtri[d].size();
        L.ea_cols[0] = (int32_t *)(C.d_lists + off[d].ea[0]);
        L.ea_cols[1] = (int32_t *)(C.d_lists + off[d].ea[1]);
        L.nea[0] = (int64_t)ea0[d].size() / 2;
        L.nea[1] = (int64_t)ea1[d].size() / 2;
        L.asm_dst = (int64_t *)(C.d_lists + off[d].dst);
        L.asm_val = (double *)(C.d_lists + off[d].val);
        L.nasm = (int64_t)adst[d].size();
    }
    DCHK(hipMalloc((void **)&C.d_panel, sizeof(double) * std::max<int64_t>(panel, 1)));
    C.stats.factor_mb = panel * 8e-6;
    return FEMCG_OK;
}

// Numeric factorisation on stream s (panels and update blocks zeroed level by
// level, A entries, extend-add, partial Cholesky); synchronises.
int chol_numeric(fem_chol &C, hipStream_t s)
{
    double *ubuf[2] = {nullptr, nullptr};
    int32_t *info = nullptr;
    struct Release {
        double **u;
        int32_t **i;
        ~Release()
        {
            if (u[0]) (void)hipFree(u[0]);
            if (u[1]) (void)hipFree(u[1]);
            if (*i) (void)hipFree(*i);
        }
    } release{ubuf, &info};
    for (int b = 0; b < 2; ++b) DCHK(hipMalloc((void **)&ubuf[b], sizeof(double) * std::max<int64_t>(C.max_udoubles, 1)));
    int64_t nbig = 0;
    for (const auto &L : C.lev) nbig += (int64_t)L.big.size();
    // info[i]: POTRF of the i-th larger front, info[nbig + i]: its TRTRI
    DCHK(hipMalloc((void **)&info, sizeof(int32_t) * std::max<int64_t>(2 * nbig, 1)));
    DCHK(hipMemsetAsync(info, 0, sizeof(int32_t) * std::max<int64_t>(2 * nbig, 1), s));
    DCHK(hipMemsetAsync(C.d_fail, 0, sizeof(int32_t), s));
    BCHK(rocblas_set_stream(C.blas, s));
    BCHK(rocblas_set_pointer_mode(C.blas, rocblas_pointer_mode_host));
    DCHK(hipFuncSetAttribute((const void *)k_mid_inv, hipFuncAttributeMaxDynamicSharedMemorySize,
                             (int)(sizeof(double) * kMidFront * kPanel)));
    const int nlev = (int)C.lev.size();
    int64_t ib = 0;
    for (int d = nlev - 1; d >= 0; --d) {
        const fem_chol::Level &L = C.lev[d];
        double *u = ubuf[d & 1];
        const double *uc = ubuf[(d + 1) & 1];
        DCHK(hipMemsetAsync(C.d_panel + L.panel0, 0, sizeof(double) * (L.panel1 - L.panel0), s));
        if (L.udoubles) DCHK(hipMemsetAsync(u, 0, sizeof(double) * L.udoubles, s));
        if (L.nasm) hipLaunchKernelGGL(k_assemble, dim3(dgrid(L.nasm)), dim3(kDBlock), 0, s, L.asm_dst, L.asm_val, L.nasm, C.d_panel);
        for (int sl = 0; sl < 2; ++sl)
            if (L.nea[sl])
                hipLaunchKernelGGL(k_extend_add, dim3((unsigned)L.nea[sl]), dim3(kDBlock), 0, s, C.d_nodes, L.ea_cols[sl],
                                   sl, C.d_index, C.d_panel, u, uc);
        if (L.nmid) {
            hipLaunchKernelGGL(k_mid_factor, dim3(L.nmid), dim3(kDBlock), 0, s, C.d_nodes, L.mid, C.d_panel, C.d_fail, 0);
            if (L.mid_tiles)
                hipLaunchKernelGGL((k_mid_update<kSyT, kSyK>), dim3(L.nmid, L.mid_tiles), dim3(kDBlock), 0, s,
                                   C.d_nodes, L.mid, C.d_panel, u);
        }
        if (L.nbigtri) {
            // own block, L11^-1 (and its transpose), L21 = F21 L11^-T, U -= L21 L21^T
            hipLaunchKernelGGL(k_mid_factor, dim3(L.nbigtri), dim3(kDBlock), 0, s, C.d_nodes, L.dbigtri, C.d_panel,
                               C.d_fail, 1);
            hipLaunchKernelGGL(k_mid_inv, dim3(L.nbigtri), dim3(kDBlock), sizeof(double) * kMidFront * kPanel, s,
                               C.d_nodes, L.dbigtri, C.d_panel);
            if (L.tri_rowtiles)
                hipLaunchKernelGGL(k_mid_l21, dim3(L.nbigtri, L.tri_rowtiles), dim3(kDBlock), 0, s, C.d_nodes, L.dbigtri,
                                   C.d_panel);
            if (L.tri_tiles)
                hipLaunchKernelGGL((k_mid_update<kTriT, kTriK>), dim3(L.nbigtri, L.tri_tiles), dim3(kDBlock), 0, s,
                                   C.d_nodes, L.dbigtri, C.d_panel, u);
        }
        DCHK(hipGetLastError());
        for (int32_t k : L.big) {
            const DNode &D = C.hnodes[k];
            const int f = D.no + D.nu;
            double *P = C.d_panel + D.panel;
            if (own_path(D.no, D.nu)) {
                ++ib;
                continue;
            }
            if (D.no > kMidFront) BCHK(rocsolver_dpotrf(C.blas, rocblas_fill_lower, D.no, P, f, info + ib));
            if (D.no > 0 && D.nu > 0) {
                const double one = 1.0, mone = -1.0;
                BCHK(rocblas_dtrsm(C.blas, rocblas_side_right, rocblas_fill_lower, rocblas_operation_transpose,
                                   rocblas_diagonal_non_unit, D.nu, D.no, &one, P, f, P + D.no, f));
                BCHK(rocblas_dsyrk(C.blas, rocblas_fill_lower, rocblas_operation_none, D.nu, D.no, &mone, P + D.no, f,
                                   &one, u + D.u, D.nu));
            }
            // L11 -> L11^-1 for the product-form solves (L21 and U no longer need L11)
            if (D.no > 0)
                BCHK(rocsolver_dtrtri(C.blas, rocblas_fill_lower, rocblas_diagonal_non_unit, D.no, P, f, info + nbig + ib));
            ++ib;
        }
    }
    // the own blocks of the fronts up to kMidFront inverted in place
    for (const auto &L : C.lev)
        if (L.nmid) {
            const int lds = std::max(L.mid_rows * kPanel, (kMirrorTile / 2) * (kMirrorTile / 2 + 1));
            hipLaunchKernelGGL(k_mid_inv, dim3(L.nmid), dim3(kDBlock), sizeof(double) * lds, s, C.d_nodes, L.mid,
                               C.d_panel);
        }
    // the larger fronts' L11^-1 mirrored into their upper triangles (the
    // grid walks the tile list in slices of at most 2^20 workgroups)
    for (int64_t m0 = 0; m0 < C.nmir; m0 += (int64_t)1 << 20) {
        const int64_t m = std::min<int64_t>(C.nmir - m0, (int64_t)1 << 20);
        hipLaunchKernelGGL(k_mirror, dim3((unsigned)m), dim3(kDBlock), 0, s, C.d_nodes, C.d_mir + 2 * m0, C.d_panel);
    }
    DCHK(hipGetLastError());
    DCHK(hipStreamSynchronize(s));
    int32_t bad = 0;
    DCHK(hipMemcpy(&bad, C.d_fail, sizeof bad, hipMemcpyDeviceToHost));
    if (nbig) {
        std::vector<int32_t> h(2 * nbig);
        DCHK(hipMemcpy(h.data(), info, sizeof(int32_t) * 2 * nbig, hipMemcpyDeviceToHost));
        for (int32_t v : h) bad |= v != 0;
    }
    if (bad) return fail(FEMCG_EBREAKDOWN, "chol_factor: non-positive pivot (A not positive definite)");
    return FEMCG_OK;
}

// One product-form step of the larger fronts of a level: q = 0..3 as in
// Level::prod, right-hand-side columns in chunks of TC.
template <int TC>
static void launch_prod(const fem_chol &C, const fem_chol::Level &L, int q, double *z, int t, double *w, hipStream_t s)
{
    if (!L.nprod[q]) return;
    const dim3 grid((unsigned)L.nprod[q], (unsigned)((t + TC - 1) / TC));
    if (q == 1)
        hipLaunchKernelGGL(k_big_rows<TC>, grid, dim3(kDBlock), 0, s, C.d_nodes, L.prod[q], C.d_panel, z, t, w);
    else
        hipLaunchKernelGGL(k_big_cols<TC>, grid, dim3(kDBlock), 0, s, C.d_nodes, L.prod[q],
                           q == 0 ? kUp : (q == 2 ? kL21 : kLow), C.d_panel, z, t, w);
}

// Right-hand-side columns per workgroup of a level's fronts up to
// kMidFront: as many as the LDS holds for its largest front.
static int mid_chunk(const fem_chol::Level &L, int t)
{
    return std::max(1, std::min(t, kSolveLds / std::max<int>(L.solve_rows, 1)));
}

static void prod_step(const fem_chol &C, const fem_chol::Level &L, int q, double *z, int t, double *w, hipStream_t s)
{
    if (t == 1) launch_prod<1>(C, L, q, z, t, w, s);
    else if (t == 2) launch_prod<2>(C, L, q, z, t, w, s);
    else if (t <= 4) launch_prod<4>(C, L, q, z, t, w, s);
    else launch_prod<8>(C, L, q, z, t, w, s);  // chunks of 8 beyond (16 measured 3% slower at t = 64)
}

// Forward and backward solve of t right-hand sides (device [n][t], public
// order) on stream s; synchronises.  Per level, fronts up to kMidFront take
// one workgroup per column chunk (gather, products with L11^-1 and L21,
// store); the larger fronts are gathered, then go through the four
// product steps.
int chol_solve_impl(fem_chol &C, const double *B, double *X, int t, hipStream_t s)
{
    const int64_t n = C.n;
    double *z = nullptr, *wb[2] = {nullptr, nullptr};
    struct Release {
        double **z, **w;
        ~Release()
        {
            if (*z) (void)hipFree(*z);
            if (w[0]) (void)hipFree(w[0]);
            if (w[1]) (void)hipFree(w[1]);
        }
    } release{&z, wb};
    DCHK(hipMalloc((void **)&z, sizeof(double) * std::max<int64_t>(n * t, 1)));
    for (int b = 0; b < 2; ++b) DCHK(hipMalloc((void **)&wb[b], sizeof(double) * std::max<int64_t>(C.max_wunits * t, 1)));
    const size_t kSolveBytes = sizeof(double) * kSolveLds;
    for (const void *fn : {(const void *)k_mid_fwd, (const void *)k_mid_bwd})
        DCHK(hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)kSolveBytes));
    hipLaunchKernelGGL(k_permute, dim3(dgrid(n * t)), dim3(kDBlock), 0, s, C.d_perm, n, t, B, z, 1);
    const int nlev = (int)C.lev.size();
    for (int d = nlev - 1; d >= 0; --d) {
        const fem_chol::Level &L = C.lev[d];
        double *w = wb[d & 1];
        const double *wc = wb[(d + 1) & 1];
        if (L.nmid) {
            const int cw = mid_chunk(L, t);
            hipLaunchKernelGGL(k_mid_fwd, dim3(L.nmid, (t + cw - 1) / cw), dim3(kDBlock), kSolveBytes, s, C.d_nodes, L.mid,
                               C.d_index, C.d_panel, z, t, cw, w, wc);
        }
        if (!L.big.empty()) {
            hipLaunchKernelGGL(k_big_fwd_gather, dim3((unsigned)L.nprod[4]), dim3(kDBlock), 0, s, C.d_nodes, L.prod[4],
                               C.d_index, z, t, w, wc);
            prod_step(C, L, 0, z, t, w, s);  // y = L11^-1 w_own -> z (columns of the mirror)
            prod_step(C, L, 1, z, t, w, s);  // w_upd -= L21 y
        }
        DCHK(hipGetLastError());
    }
    for (int d = 0; d < nlev; ++d) {
        const fem_chol::Level &L = C.lev[d];
        double *w = wb[0];
        if (L.nmid) {
            const int cw = mid_chunk(L, t);
            hipLaunchKernelGGL(k_mid_bwd, dim3(L.nmid, (t + cw - 1) / cw), dim3(kDBlock), kSolveBytes, s, C.d_nodes, L.mid,
                               C.d_index, C.d_panel, z, t, cw);
        }
        if (!L.big.empty()) {
            hipLaunchKernelGGL(k_big_bwd_gather, dim3((unsigned)L.nprod[4]), dim3(kDBlock), 0, s, C.d_nodes, L.prod[4],
                               C.d_index, z, t, w);
            prod_step(C, L, 2, z, t, w, s);  // w_own -= L21^T x_upd
            prod_step(C, L, 3, z, t, w, s);  // x = L11^-T w_own -> z
        }
        DCHK(hipGetLastError());
    }
    hipLaunchKernelGGL(k_permute, dim3(dgrid(n * t)), dim3(kDBlock), 0, s, C.d_perm, n, t, z, X, 0);
    DCHK(hipGetLastError());
    DCHK(hipStreamSynchronize(s));
    return FEMCG_OK;
}

}  // namespace femcg

using namespace femcg;

fem_chol::~fem_chol()
{
    if (d_nodes) (void)hipFree(d_nodes);
    if (d_perm) (void)hipFree(d_perm);
    if (d_index) (void)hipFree(d_index);
    if (d_panel) (void)hipFree(d_panel);
    if (d_lists) (void)hipFree(d_lists);
    if (d_fail) (void)hipFree(d_fail);
    if (blas) (void)rocblas_destroy_handle(blas);
}

extern "C" int chol_analyze(const fem_matrix *A, chol_stats_t *out, int32_t *perm_out)
{
    if (!A || !out) return fail(FEMCG_EINVAL, "NULL argument");
    try {
        fem_chol C;
        int rc = chol_symbolic(A->hs, C);
        if (rc) return rc;
        *out = C.stats;
        if (perm_out) std::copy(C.perm.begin(), C.perm.end(), perm_out);
        return FEMCG_OK;
    } catch (const std::bad_alloc &) {
        return fail(FEMCG_ENOMEM, "chol_analyze: host allocation failed");
    } catch (const std::exception &ex) {  // e.g. no host thread for the ordering
        return fail(FEMCG_ENOMEM, "chol_analyze: %s", ex.what());
    }
}

extern "C" int chol_factor(fem_matrix *A, fem_chol **out, void *stream)
{
    if (!A || !out) return fail(FEMCG_EINVAL, "NULL argument");
    *out = nullptr;
    if (int rc = require_device(A)) return rc;
    try {
        const double t0 = now_s();
        auto C = std::make_unique<fem_chol>();
        int rc = chol_symbolic(A->hs, *C);
        if (rc) return rc;
        const double t1 = now_s();
        if ((rc = chol_setup(A->hs, *C))) return rc;
        if (rocblas_create_handle(&C->blas) != rocblas_status_success)
            return fail(FEMCG_EDEVICE, "rocblas_create_handle failed");
        const double t2 = now_s();
        if ((rc = chol_numeric(*C, (hipStream_t)stream))) return rc;
        const double t3 = now_s();
        C->stats.symbolic_s += t2 - t1;  // host set-up and uploads belong to the symbolic phase
        C->stats.factor_s = t3 - t2;
        C->stats.total_s = t3 - t0;
        *out = C.release();
        return FEMCG_OK;
    } catch (const std::bad_alloc &) {
        return fail(FEMCG_ENOMEM, "chol_factor: host allocation failed");
    } catch (const std::exception &ex) {  // e.g. no host thread for the ordering
        return fail(FEMCG_ENOMEM, "chol_factor: %s", ex.what());
    }
}

extern "C" int chol_solve(fem_chol *L, const double *B, double *X, int32_t k, void *stream)
{
    if (!L || !B || !X) return fail(FEMCG_EINVAL, "NULL argument");
    if (k < 1) return fail(FEMCG_EINVAL, "k=%d", k);
    try {
        const double t0 = now_s();
        int rc = chol_solve_impl(*L, B, X, k, (hipStream_t)stream);
        L->stats.solve_s = now_s() - t0;
        return rc;
    } catch (const std::bad_alloc &) {
        return fail(FEMCG_ENOMEM, "chol_solve: host allocation failed");
    } catch (const std::exception &ex) {  // e.g. no host thread for the ordering
        return fail(FEMCG_ENOMEM, "chol_solve: %s", ex.what());
    }
}

extern "C" int chol_stats(const fem_chol *L, chol_stats_t *out)
{
    if (!L || !out) return fail(FEMCG_EINVAL, "NULL argument");
    *out = L->stats;
    return FEMCG_OK;
}

extern "C" void chol_free(fem_chol *L)
{
    delete L;
}
