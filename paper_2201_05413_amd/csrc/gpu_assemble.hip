// gpu_assemble.hip -- FEM assembly on the device (mesh -> A = K_II and the
// lifting operator K_ID), the same result as assemble_host.
//
// The stiffness matrix is the element-by-element sum of Sect. 2.2's local
// matrices (closed forms in element.h).  On the device:
//   1. Edges (P2-P4): sort the (min, max) vertex-pair keys of every cell
//      edge, unique -> the edges in (min, max) order; each cell's edge DOFs by
//      binary search (P3/P4: p-1 per edge, oriented from the smaller vertex,
//      then the cell's interior DOFs).
//   2. Dirichlet DOFs: boundary vertices as flagged; an edge's DOFs are
//      Dirichlet if it lies on a boundary facet (a facet of exactly one cell:
//      run-length encoding of the sorted facet keys) whose vertices are all
//      flagged.
//   3. Free / Dirichlet numbering: exclusive scans of the flags.
//   4. Element matrices, one thread per cell (P3/P4: from the host's
//      geometry-free moment table, K = |T| sum_mn (g_m . g_n) M^mn).
//   5. Every entry K_e[a][b] of a free row becomes the pair (row, col) -> value;
//      a stable radix sort by (row, col) keeps equal keys in cell order, and
//      each run is summed sequentially in that order (the summation order of
//      the reference assembly).
//   6. Runs split into A (free columns, free numbering) and K_ID (Dirichlet
//      columns, Dirichlet numbering); row pointers from the first run of each
//      row.
// The results are copied into the HostSystem, so every host-side consumer
// (solver copy, lifting upload, DOF queries) is unchanged.
#include <hipcub/hipcub.hpp>

#include <algorithm>
#include <cstring>
#include <vector>

#include "assemble.h"
#include "element.h"

namespace femcg {

namespace {

constexpr int kTpb = 256;

inline unsigned blocks_for(int64_t n) { return (unsigned)std::max<int64_t>(1, (n + kTpb - 1) / kTpb); }

// device buffers released on scope exit
struct DevBufs {
    std::vector<void *> ptrs;
    ~DevBufs()
    {
        for (void *p : ptrs) (void)hipFree(p);
    }
    template <typename T>
    hipError_t alloc(T **p, size_t count)
    {
        *p = nullptr;
        hipError_t e = hipMalloc((void **)p, std::max<size_t>(count, 1) * sizeof(T));
        if (e == hipSuccess) ptrs.push_back(*p);
        return e;
    }
};

__global__ void k_edge_keys(const int32_t *__restrict__ cells, int64_t nc, int nvl, int nel, uint64_t *__restrict__ keys)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nc * nel) return;
    int E[6][2];
    local_edges(nvl - 1, E);
    const int64_t c = i / nel;
    const int e = (int)(i % nel);
    uint64_t a = (uint32_t)cells[c * nvl + E[e][0]], b = (uint32_t)cells[c * nvl + E[e][1]];
    if (a > b) {
        const uint64_t t = a;
        a = b;
        b = t;
    }
    keys[i] = (a << 32) | b;
}

__device__ __forceinline__ int64_t lower_bound_u64(const uint64_t *__restrict__ v, int64_t n, uint64_t key)
{
    int64_t lo = 0, hi = n;
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (v[mid] < key) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

__global__ void k_cell_dofs(const int32_t *__restrict__ cells, const uint64_t *__restrict__ ekeys,
                            const uint64_t *__restrict__ edges, int64_t nedges, int64_t nc, int nvl, int nel,
                            int nl, int64_t nv, int order, int64_t ibase, int32_t *__restrict__ cdofs)
{
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= nc) return;
    for (int i = 0; i < nvl; ++i) cdofs[c * nl + i] = cells[c * nvl + i];
    if (order == 2) {
        for (int e = 0; e < nel; ++e)
            cdofs[c * nl + nvl + e] = (int32_t)(nv + lower_bound_u64(edges, nedges, ekeys[c * nel + e]));
    } else if (order >= 3) {
        // triangles: edge e = (la, lb) holds its points s = 1..p-1 from la on;
        // the global DOF t (1..p-1) counts from the edge's smaller vertex
        const int ke = order - 1, ci = (order - 1) * (order - 2) / 2;
        int E[6][2];
        local_edges(2, E);
        for (int e = 0; e < 3; ++e) {
            const int64_t idx = lower_bound_u64(edges, nedges, ekeys[c * 3 + e]);
            const int32_t va = cells[c * 3 + E[e][0]], vb = cells[c * 3 + E[e][1]];
            for (int s = 1; s < order; ++s) {
                const int t = va > vb ? order - s : s;
                cdofs[c * nl + 3 + e * ke + (s - 1)] = (int32_t)(nv + ke * idx + t - 1);
            }
        }
        for (int r = 0; r < ci; ++r) cdofs[c * nl + 3 + 3 * ke + r] = (int32_t)(ibase + ci * c + r);
    }
}

__global__ void k_vertex_flags(const uint8_t *__restrict__ bnd, int64_t nv, uint8_t *__restrict__ dir)
{
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v < nv) dir[v] = bnd[v] ? 1 : 0;
}

// 2D P2-P4: an edge of exactly one triangle with both ends flagged (its ke DOFs)
__global__ void k_dir_edges_2d(const uint64_t *__restrict__ ukeys, const int32_t *__restrict__ counts, int64_t nrun,
                               const uint8_t *__restrict__ bnd, const uint64_t *__restrict__ edges, int64_t nedges,
                               int64_t nv, int ke, uint8_t *__restrict__ dir)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nrun || counts[i] != 1) return;
    const uint64_t k = ukeys[i];
    if (bnd[k >> 32] && bnd[k & 0xffffffffu]) {
        const int64_t idx = lower_bound_u64(edges, nedges, k);
        for (int t = 0; t < ke; ++t) dir[nv + ke * idx + t] = 1;
    }
}

// 3D: face keys (sorted vertex triple, 21 bits each)
__global__ void k_face_keys(const int32_t *__restrict__ cells, int64_t nc, uint64_t *__restrict__ keys)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nc * 4) return;
    const int64_t c = i / 4;
    const int o = (int)(i % 4);
    uint32_t v[3];
    int q = 0;
    for (int t = 0; t < 4; ++t)
        if (t != o) v[q++] = (uint32_t)cells[c * 4 + t];
    if (v[0] > v[1]) { const uint32_t t = v[0]; v[0] = v[1]; v[1] = t; }
    if (v[1] > v[2]) { const uint32_t t = v[1]; v[1] = v[2]; v[2] = t; }
    if (v[0] > v[1]) { const uint32_t t = v[0]; v[0] = v[1]; v[1] = t; }
    keys[i] = ((uint64_t)v[0] << 42) | ((uint64_t)v[1] << 21) | (uint64_t)v[2];
}

__global__ void k_dir_edges_3d(const uint64_t *__restrict__ ukeys, const int32_t *__restrict__ counts, int64_t nrun,
                               const uint8_t *__restrict__ bnd, const uint64_t *__restrict__ edges, int64_t nedges,
                               int64_t nv, uint8_t *__restrict__ dir)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nrun || counts[i] != 1) return;
    const uint64_t k = ukeys[i];
    const uint64_t m = (1ull << 21) - 1;
    const uint64_t v[3] = {k >> 42, (k >> 21) & m, k & m};
    if (!(bnd[v[0]] && bnd[v[1]] && bnd[v[2]])) return;
    const int pr[3][2] = {{0, 1}, {0, 2}, {1, 2}};
    for (int p = 0; p < 3; ++p) {
        const uint64_t key = (v[pr[p][0]] << 32) | v[pr[p][1]];
        dir[nv + lower_bound_u64(edges, nedges, key)] = 1;
    }
}

__global__ void k_flags_to_int(const uint8_t *__restrict__ dir, int64_t n, int32_t *__restrict__ isfree,
                               int32_t *__restrict__ isdir)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    isfree[i] = dir[i] ? 0 : 1;
    isdir[i] = dir[i] ? 1 : 0;
}

// element matrices + the (free row, column DOF) keys of their entries;
// entries of Dirichlet rows get the key ~0 (sorted last, dropped)
__global__ void k_elements(const double *__restrict__ coords, const int32_t *__restrict__ cells,
                           const int32_t *__restrict__ cdofs, const uint8_t *__restrict__ dir,
                           const int32_t *__restrict__ fscan, int64_t nc, int dim, int order, int nl,
                           const double *__restrict__ pkM, uint64_t *__restrict__ keys, double *__restrict__ vals,
                           unsigned *__restrict__ nbad)
{
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= nc) return;
    const int nvl = dim + 1;
    double P[12];
    for (int i = 0; i < nvl; ++i)
        for (int r = 0; r < dim; ++r) P[i * dim + r] = coords[(int64_t)cells[c * nvl + i] * dim + r];
    if (order >= 3) {
        // P3/P4 triangles: entry (a, b) = sum_mn |T| (g_m . g_n) M^mn_ab,
        // summed over m, n in the host's order
        double g[4][3] = {}, area;
        if (!simplex_grads(2, P, g, &area)) {
            atomicAdd(nbad, 1u);
            for (int t = 0; t < nl * nl; ++t) {
                keys[c * nl * nl + t] = ~0ull;
                vals[c * nl * nl + t] = 0.0;
            }
            return;
        }
        double G[9];
        for (int m = 0; m < 3; ++m)
            for (int n = 0; n < 3; ++n) G[m * 3 + n] = area * (g[m][0] * g[n][0] + g[m][1] * g[n][1]);
        const int64_t nl2 = (int64_t)nl * nl;
        for (int a = 0; a < nl; ++a) {
            const int32_t ra = cdofs[c * nl + a];
            const bool free_row = dir[ra] == 0;
            const uint64_t rk = (uint64_t)(uint32_t)fscan[ra] << 32;
            for (int b = 0; b < nl; ++b) {
                double v = 0.0;
                for (int mn = 0; mn < 9; ++mn) v += G[mn] * pkM[mn * nl2 + a * nl + b];
                const int64_t o = c * nl2 + a * nl + b;
                keys[o] = free_row ? (rk | (uint32_t)cdofs[c * nl + b]) : ~0ull;
                vals[o] = v;
            }
        }
        return;
    }
    double K[100];
    if (!element_matrix(dim, order, P, K)) {
        atomicAdd(nbad, 1u);
        for (int t = 0; t < nl * nl; ++t) {
            keys[c * nl * nl + t] = ~0ull;
            vals[c * nl * nl + t] = 0.0;
        }
        return;
    }
    for (int a = 0; a < nl; ++a) {
        const int32_t ra = cdofs[c * nl + a];
        const bool free_row = dir[ra] == 0;
        const uint64_t rk = (uint64_t)(uint32_t)fscan[ra] << 32;
        for (int b = 0; b < nl; ++b) {
            const int64_t o = c * nl * nl + a * nl + b;
            keys[o] = free_row ? (rk | (uint32_t)cdofs[c * nl + b]) : ~0ull;
            vals[o] = K[a * nl + b];
        }
    }
}

__global__ void k_run_heads(const uint64_t *__restrict__ keys, int64_t n, int32_t *__restrict__ head)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    head[i] = (keys[i] != ~0ull && (i == 0 || keys[i] != keys[i - 1])) ? 1 : 0;
}

__global__ void k_run_starts(const int32_t *__restrict__ head, const int64_t *__restrict__ hscan, int64_t n,
                             int64_t *__restrict__ start)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n && head[i]) start[hscan[i]] = i;
}

// one thread per run: the sum of its entries in cell order, and whether the
// column is free (A) or Dirichlet (K_ID)
__global__ void k_run_sums(const uint64_t *__restrict__ keys, const double *__restrict__ vals,
                           const int64_t *__restrict__ start, int64_t nrun, int64_t nent,
                           const uint8_t *__restrict__ dir, double *__restrict__ sum, int32_t *__restrict__ isa,
                           int32_t *__restrict__ isl)
{
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= nrun) return;
    const int64_t b = start[r];
    const int64_t e = r + 1 < nrun ? start[r + 1] : nent;
    double s = 0.0;
    for (int64_t t = b; t < e; ++t) s += vals[t];
    sum[r] = s;
    const uint32_t cd = (uint32_t)(keys[b] & 0xffffffffu);
    isa[r] = dir[cd] ? 0 : 1;
    isl[r] = dir[cd] ? 1 : 0;
}

__global__ void k_split(const uint64_t *__restrict__ keys, const int64_t *__restrict__ start, const double *__restrict__ sum,
                        const int32_t *__restrict__ isa, const int64_t *__restrict__ ascan,
                        const int64_t *__restrict__ lscan, int64_t nrun, const int32_t *__restrict__ fscan,
                        const int32_t *__restrict__ dscan, int32_t *__restrict__ acol, double *__restrict__ aval,
                        int32_t *__restrict__ lcol, double *__restrict__ lval, int64_t *__restrict__ arow,
                        int64_t *__restrict__ lrow)
{
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= nrun) return;
    const uint64_t k = keys[start[r]];
    const uint32_t row = (uint32_t)(k >> 32), cd = (uint32_t)(k & 0xffffffffu);
    if (isa[r]) {
        acol[ascan[r]] = fscan[cd];
        aval[ascan[r]] = sum[r];
    } else {
        lcol[lscan[r]] = dscan[cd];
        lval[lscan[r]] = sum[r];
    }
    if (r == 0 || (uint32_t)(keys[start[r - 1]] >> 32) != row) {
        arow[row] = ascan[r];
        lrow[row] = lscan[r];
    }
}

}  // namespace

#define DCHK(call)                                                                     \
    do {                                                                               \
        hipError_t e_ = (call);                                                        \
        if (e_ != hipSuccess) {                                                        \
            err = std::string(#call) + ": " + hipGetErrorString(e_);                   \
            return e_ == hipErrorOutOfMemory ? FEMCG_ENOMEM : FEMCG_EDEVICE;           \
        }                                                                              \
    } while (0)

int assemble_device(const fem_mesh *mesh, int order, HostSystem &hs, std::string &err, hipStream_t s)
{
    const int dim = mesh->dim;
    if ((dim != 2 && dim != 3) || order < 1 || order > 4 || (order > 2 && dim != 2)) {
        err = "unsupported dimension or order";
        return FEMCG_EUNSUPPORTED;
    }
    if (mesh->nverts <= 0 || mesh->ncells <= 0 || !mesh->coords || !mesh->cells || !mesh->on_boundary) {
        err = "empty mesh or NULL array";
        return FEMCG_EINVAL;
    }
    const int64_t nv = mesh->nverts, nc = mesh->ncells;
    const int nvl = dim + 1;
    int E[6][2];
    const int nel = local_edges(dim, E);
    const int nl = order == 1 ? nvl : (order == 2 ? nvl + nel : (order + 1) * (order + 2) / 2);
    const int ke = order - 1, ci = (order - 1) * (order - 2) / 2;  // DOFs per edge, per cell interior
    // index ranges of the device path: 21-bit face keys (3D P2), 32-bit DOFs,
    // int item counts of the device-wide sorts and scans
    if ((dim == 3 && order == 2 && nv >= ((int64_t)1 << 21)) || nv >= ((int64_t)1 << 30) ||
        nc * nl * nl >= ((int64_t)1 << 31) - 1 || nc * 4 >= ((int64_t)1 << 31) - 1) {
        err = "mesh beyond the device assembly's index ranges";
        return FEMCG_EUNSUPPORTED;
    }
    for (int64_t i = 0; i < nc * nvl; ++i)
        if (mesh->cells[i] < 0 || mesh->cells[i] >= nv) {
            err = "cell vertex index out of range";
            return FEMCG_EMESH;
        }
    hs.dim = dim;
    hs.order = order;
    hs.nverts = nv;
    hs.ncells = nc;
    hs.nloc = nl;
    DevBufs buf;
    double *d_coords;
    int32_t *d_cells;
    uint8_t *d_bnd;
    DCHK(buf.alloc(&d_coords, (size_t)nv * dim));
    DCHK(buf.alloc(&d_cells, (size_t)nc * nvl));
    DCHK(buf.alloc(&d_bnd, (size_t)nv));
    DCHK(hipMemcpyAsync(d_coords, mesh->coords, sizeof(double) * nv * dim, hipMemcpyHostToDevice, s));
    DCHK(hipMemcpyAsync(d_cells, mesh->cells, sizeof(int32_t) * nc * nvl, hipMemcpyHostToDevice, s));
    DCHK(hipMemcpyAsync(d_bnd, mesh->on_boundary, nv, hipMemcpyHostToDevice, s));
    size_t tmp_bytes = 0;
    void *d_tmp = nullptr;
    auto need_tmp = [&](size_t bytes) -> hipError_t {
        if (bytes <= tmp_bytes) return hipSuccess;
        if (d_tmp) {
            (void)hipFree(d_tmp);
            buf.ptrs.erase(std::find(buf.ptrs.begin(), buf.ptrs.end(), d_tmp));
            d_tmp = nullptr;
        }
        tmp_bytes = bytes;
        return buf.alloc((char **)&d_tmp, bytes);
    };
    int64_t *d_count;  // device scalar outputs of select / run-length passes
    DCHK(buf.alloc(&d_count, 1));

    // ---- 1. edges ----
    uint64_t *d_ekey = nullptr, *d_esort = nullptr, *d_edges = nullptr;
    int64_t nedges = 0;
    const int64_t ne_all = order >= 2 ? nc * nel : 0;
    if (order >= 2) {
        DCHK(buf.alloc(&d_ekey, ne_all));
        DCHK(buf.alloc(&d_esort, ne_all));
        DCHK(buf.alloc(&d_edges, ne_all));
        hipLaunchKernelGGL(k_edge_keys, dim3(blocks_for(ne_all)), dim3(kTpb), 0, s, d_cells, nc, nvl, nel, d_ekey);
        size_t tb = 0;
        DCHK(hipcub::DeviceRadixSort::SortKeys(nullptr, tb, d_ekey, d_esort, (int)ne_all, 0, 64, s));
        DCHK(need_tmp(tb));
        DCHK(hipcub::DeviceRadixSort::SortKeys(d_tmp, tb, d_ekey, d_esort, (int)ne_all, 0, 64, s));
        DCHK(hipcub::DeviceSelect::Unique(nullptr, tb, d_esort, d_edges, d_count, (int)ne_all, s));
        DCHK(need_tmp(tb));
        DCHK(hipcub::DeviceSelect::Unique(d_tmp, tb, d_esort, d_edges, d_count, (int)ne_all, s));
        DCHK(hipMemcpyAsync(&nedges, d_count, sizeof(int64_t), hipMemcpyDeviceToHost, s));
        DCHK(hipStreamSynchronize(s));
    }
    hs.nedges = nedges;
    hs.ndofs = nv + ke * nedges + (int64_t)ci * nc;
    const int64_t nd = hs.ndofs;
    if (nd >= ((int64_t)1 << 31)) {
        err = "too many DOFs for int32 indices";
        return FEMCG_EUNSUPPORTED;
    }
    int32_t *d_cdofs;
    DCHK(buf.alloc(&d_cdofs, (size_t)nc * nl));
    hipLaunchKernelGGL(k_cell_dofs, dim3(blocks_for(nc)), dim3(kTpb), 0, s, d_cells, d_ekey, d_edges, nedges, nc, nvl,
                       nel, nl, nv, order, (int64_t)(nv + ke * nedges), d_cdofs);

    // ---- 2. Dirichlet flags ----
    uint8_t *d_dir;
    DCHK(buf.alloc(&d_dir, (size_t)nd));
    DCHK(hipMemsetAsync(d_dir, 0, nd, s));
    hipLaunchKernelGGL(k_vertex_flags, dim3(blocks_for(nv)), dim3(kTpb), 0, s, d_bnd, nv, d_dir);
    if (order >= 2) {
        const int64_t nf_all = dim == 2 ? ne_all : nc * 4;
        uint64_t *d_fkey = d_esort;  // 2D: the sorted edge keys are the facet keys
        uint64_t *d_uk;
        int32_t *d_cnt;
        DCHK(buf.alloc(&d_uk, nf_all));
        DCHK(buf.alloc(&d_cnt, nf_all));
        if (dim == 3) {
            uint64_t *d_fraw;
            DCHK(buf.alloc(&d_fraw, nf_all));
            DCHK(buf.alloc(&d_fkey, nf_all));
            hipLaunchKernelGGL(k_face_keys, dim3(blocks_for(nf_all)), dim3(kTpb), 0, s, d_cells, nc, d_fraw);
            size_t tb = 0;
            DCHK(hipcub::DeviceRadixSort::SortKeys(nullptr, tb, d_fraw, d_fkey, (int)nf_all, 0, 63, s));
            DCHK(need_tmp(tb));
            DCHK(hipcub::DeviceRadixSort::SortKeys(d_tmp, tb, d_fraw, d_fkey, (int)nf_all, 0, 63, s));
        }
        size_t tb = 0;
        DCHK(hipcub::DeviceRunLengthEncode::Encode(nullptr, tb, d_fkey, d_uk, d_cnt, d_count, (int)nf_all, s));
        DCHK(need_tmp(tb));
        DCHK(hipcub::DeviceRunLengthEncode::Encode(d_tmp, tb, d_fkey, d_uk, d_cnt, d_count, (int)nf_all, s));
        int64_t nrun = 0;
        DCHK(hipMemcpyAsync(&nrun, d_count, sizeof(int64_t), hipMemcpyDeviceToHost, s));
        DCHK(hipStreamSynchronize(s));
        if (dim == 2)
            hipLaunchKernelGGL(k_dir_edges_2d, dim3(blocks_for(nrun)), dim3(kTpb), 0, s, d_uk, d_cnt, nrun, d_bnd,
                               d_edges, nedges, nv, ke, d_dir);
        else
            hipLaunchKernelGGL(k_dir_edges_3d, dim3(blocks_for(nrun)), dim3(kTpb), 0, s, d_uk, d_cnt, nrun, d_bnd,
                               d_edges, nedges, nv, d_dir);
    }

    // ---- 3. numbering ----
    int32_t *d_isf, *d_isd, *d_fscan, *d_dscan;
    DCHK(buf.alloc(&d_isf, nd));
    DCHK(buf.alloc(&d_isd, nd));
    DCHK(buf.alloc(&d_fscan, nd));
    DCHK(buf.alloc(&d_dscan, nd));
    hipLaunchKernelGGL(k_flags_to_int, dim3(blocks_for(nd)), dim3(kTpb), 0, s, d_dir, nd, d_isf, d_isd);
    {
        size_t tb = 0;
        DCHK(hipcub::DeviceScan::ExclusiveSum(nullptr, tb, d_isf, d_fscan, (int)nd, s));
        DCHK(need_tmp(tb));
        DCHK(hipcub::DeviceScan::ExclusiveSum(d_tmp, tb, d_isf, d_fscan, (int)nd, s));
        DCHK(hipcub::DeviceScan::ExclusiveSum(d_tmp, tb, d_isd, d_dscan, (int)nd, s));
    }

    // ---- host-side numbering (O(ndofs)) ----
    hs.dirichlet.resize(nd);
    DCHK(hipMemcpyAsync(hs.dirichlet.data(), d_dir, nd, hipMemcpyDeviceToHost, s));
    DCHK(hipStreamSynchronize(s));
    hs.dof2free.assign(nd, -1);
    hs.dof2dir.assign(nd, -1);
    hs.free2dof.clear();
    hs.dir2dof.clear();
    for (int64_t d = 0; d < nd; ++d) {
        if (hs.dirichlet[d]) {
            hs.dof2dir[d] = (int64_t)hs.dir2dof.size();
            hs.dir2dof.push_back(d);
        } else {
            hs.dof2free[d] = (int64_t)hs.free2dof.size();
            hs.free2dof.push_back(d);
        }
    }
    hs.nfree = (int64_t)hs.free2dof.size();
    hs.ndir = (int64_t)hs.dir2dof.size();
    const int64_t nf = hs.nfree;
    if (nf == 0) {
        err = "mesh has no free DOFs";
        return FEMCG_EINVAL;
    }

    // ---- 4./5. element matrices, keyed entries, stable sort ----
    const int64_t nent = nc * nl * nl;
    uint64_t *d_k0, *d_k1;
    double *d_v0, *d_v1;
    unsigned *d_bad;
    DCHK(buf.alloc(&d_k0, nent));
    DCHK(buf.alloc(&d_k1, nent));
    DCHK(buf.alloc(&d_v0, nent));
    DCHK(buf.alloc(&d_v1, nent));
    DCHK(buf.alloc(&d_bad, 1));
    DCHK(hipMemsetAsync(d_bad, 0, sizeof(unsigned), s));
    double *d_pkM = nullptr;
    if (order >= 3) {
        int nlt = 0;
        const std::vector<double> &M = pk_moment_table(order, &nlt);
        if (nlt != nl || M.size() != (size_t)9 * nl * nl) {
            err = "P3/P4 moment table size mismatch";
            return FEMCG_EDEVICE;
        }
        DCHK(buf.alloc(&d_pkM, M.size()));
        DCHK(hipMemcpyAsync(d_pkM, M.data(), sizeof(double) * M.size(), hipMemcpyHostToDevice, s));
    }
    hipLaunchKernelGGL(k_elements, dim3(blocks_for(nc)), dim3(kTpb), 0, s, d_coords, d_cells, d_cdofs, d_dir, d_fscan,
                       nc, dim, order, nl, (const double *)d_pkM, d_k0, d_v0, d_bad);
    unsigned nbad = 0;
    DCHK(hipMemcpyAsync(&nbad, d_bad, sizeof(unsigned), hipMemcpyDeviceToHost, s));
    DCHK(hipStreamSynchronize(s));
    if (nbad) {
        err = "mesh has " + std::to_string(nbad) + " cells with non-positive measure";
        return FEMCG_EMESH;
    }
    hipcub::DoubleBuffer<uint64_t> dk(d_k0, d_k1);
    hipcub::DoubleBuffer<double> dv(d_v0, d_v1);
    {
        size_t tb = 0;
        DCHK(hipcub::DeviceRadixSort::SortPairs(nullptr, tb, dk, dv, (int)nent, 0, 64, s));
        DCHK(need_tmp(tb));
        DCHK(hipcub::DeviceRadixSort::SortPairs(d_tmp, tb, dk, dv, (int)nent, 0, 64, s));
    }
    const uint64_t *keys = dk.Current();
    const double *vals = dv.Current();

    // ---- runs: heads, starts, sums ----
    int32_t *d_head = (int32_t *)dk.Alternate();  // the sort's spare buffers are free now
    int64_t *d_hscan;
    DCHK(buf.alloc(&d_hscan, nent));
    hipLaunchKernelGGL(k_run_heads, dim3(blocks_for(nent)), dim3(kTpb), 0, s, keys, nent, d_head);
    {
        size_t tb = 0;
        DCHK(hipcub::DeviceScan::ExclusiveSum(nullptr, tb, d_head, d_hscan, (int)nent, s));
        DCHK(need_tmp(tb));
        DCHK(hipcub::DeviceScan::ExclusiveSum(d_tmp, tb, d_head, d_hscan, (int)nent, s));
    }
    int64_t last_scan = 0;
    int32_t last_head = 0;
    DCHK(hipMemcpyAsync(&last_scan, d_hscan + nent - 1, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    DCHK(hipMemcpyAsync(&last_head, d_head + nent - 1, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    DCHK(hipStreamSynchronize(s));
    const int64_t nrun = last_scan + last_head;
    // runs belong to free rows; ~0 keys (Dirichlet rows) form no run
    int64_t nent_free = 0;
    {
        // entries before the first ~0 key
        std::vector<uint64_t> probe(1);
        int64_t lo = 0, hi = nent;
        while (lo < hi) {
            const int64_t mid = (lo + hi) >> 1;
            DCHK(hipMemcpyAsync(probe.data(), keys + mid, sizeof(uint64_t), hipMemcpyDeviceToHost, s));
            DCHK(hipStreamSynchronize(s));
            if (probe[0] != ~0ull) lo = mid + 1;
            else hi = mid;
        }
        nent_free = lo;
    }
    int64_t *d_start;
    double *d_sum = (double *)dv.Alternate();
    int32_t *d_isa, *d_isl;
    int64_t *d_ascan, *d_lscan;
    DCHK(buf.alloc(&d_start, nrun));
    DCHK(buf.alloc(&d_isa, nrun));
    DCHK(buf.alloc(&d_isl, nrun));
    DCHK(buf.alloc(&d_ascan, nrun));
    DCHK(buf.alloc(&d_lscan, nrun));
    hipLaunchKernelGGL(k_run_starts, dim3(blocks_for(nent)), dim3(kTpb), 0, s, d_head, d_hscan, nent, d_start);
    hipLaunchKernelGGL(k_run_sums, dim3(blocks_for(nrun)), dim3(kTpb), 0, s, keys, vals, d_start, nrun, nent_free,
                       d_dir, d_sum, d_isa, d_isl);
    {
        size_t tb = 0;
        DCHK(hipcub::DeviceScan::ExclusiveSum(nullptr, tb, d_isa, d_ascan, (int)nrun, s));
        DCHK(need_tmp(tb));
        DCHK(hipcub::DeviceScan::ExclusiveSum(d_tmp, tb, d_isa, d_ascan, (int)nrun, s));
        DCHK(hipcub::DeviceScan::ExclusiveSum(d_tmp, tb, d_isl, d_lscan, (int)nrun, s));
    }
    int64_t na = 0, nlid = 0;
    int32_t la = 0, ll = 0;
    DCHK(hipMemcpyAsync(&na, d_ascan + nrun - 1, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    DCHK(hipMemcpyAsync(&nlid, d_lscan + nrun - 1, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    DCHK(hipMemcpyAsync(&la, d_isa + nrun - 1, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    DCHK(hipMemcpyAsync(&ll, d_isl + nrun - 1, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    DCHK(hipStreamSynchronize(s));
    na += la;
    nlid += ll;

    // ---- 6. split into A and K_ID ----
    int32_t *d_acol, *d_lcol;
    double *d_aval, *d_lval;
    int64_t *d_arow, *d_lrow;
    DCHK(buf.alloc(&d_acol, na));
    DCHK(buf.alloc(&d_aval, na));
    DCHK(buf.alloc(&d_lcol, nlid));
    DCHK(buf.alloc(&d_lval, nlid));
    DCHK(buf.alloc(&d_arow, nf + 1));
    DCHK(buf.alloc(&d_lrow, nf + 1));
    hipLaunchKernelGGL(k_split, dim3(blocks_for(nrun)), dim3(kTpb), 0, s, keys, d_start, d_sum, d_isa, d_ascan, d_lscan,
                       nrun, d_fscan, d_dscan, d_acol, d_aval, d_lcol, d_lval, d_arow, d_lrow);
    DCHK(hipGetLastError());
    hs.a_rowptr.resize(nf + 1);
    hs.l_rowptr.resize(nf + 1);
    hs.a_col.resize(na);
    hs.a_val.resize(na);
    hs.l_col.resize(nlid);
    hs.l_val.resize(nlid);
    DCHK(hipMemcpyAsync(hs.a_rowptr.data(), d_arow, sizeof(int64_t) * nf, hipMemcpyDeviceToHost, s));
    DCHK(hipMemcpyAsync(hs.l_rowptr.data(), d_lrow, sizeof(int64_t) * nf, hipMemcpyDeviceToHost, s));
    if (na) {
        DCHK(hipMemcpyAsync(hs.a_col.data(), d_acol, sizeof(int32_t) * na, hipMemcpyDeviceToHost, s));
        DCHK(hipMemcpyAsync(hs.a_val.data(), d_aval, sizeof(double) * na, hipMemcpyDeviceToHost, s));
    }
    if (nlid) {
        DCHK(hipMemcpyAsync(hs.l_col.data(), d_lcol, sizeof(int32_t) * nlid, hipMemcpyDeviceToHost, s));
        DCHK(hipMemcpyAsync(hs.l_val.data(), d_lval, sizeof(double) * nlid, hipMemcpyDeviceToHost, s));
    }
    std::vector<uint64_t> edges((size_t)nedges);
    if (nedges) DCHK(hipMemcpyAsync(edges.data(), d_edges, sizeof(uint64_t) * nedges, hipMemcpyDeviceToHost, s));
    DCHK(hipStreamSynchronize(s));
    hs.a_rowptr[nf] = na;
    hs.l_rowptr[nf] = nlid;
    // DOF coordinates (the public convention, as the host assembly computes
    // them): vertices; P2 edge midpoints; P3/P4 edge point t at
    // ((p-t) x_a + t x_b) / p, then the cell interiors
    hs.dof_coords.resize((size_t)nd * dim);
    std::memcpy(hs.dof_coords.data(), mesh->coords, sizeof(double) * nv * dim);
    for (int64_t e = 0; e < nedges; ++e) {
        const int64_t a = (int64_t)(edges[e] >> 32), b = (int64_t)(edges[e] & 0xffffffffu);
        for (int r = 0; r < dim; ++r) {
            const double xa = mesh->coords[a * dim + r], xb = mesh->coords[b * dim + r];
            if (order == 2)
                hs.dof_coords[(nv + e) * dim + r] = 0.5 * (xa + xb);
            else
                for (int t = 1; t <= ke; ++t)
                    hs.dof_coords[(nv + ke * e + t - 1) * dim + r] = ((double)(order - t) * xa + (double)t * xb) / order;
        }
    }
    if (order >= 3) {
        int ia[3][3], ni = 0;  // interior barycentric indices, decreasing lexicographic order
        for (int a0 = order - 2; a0 >= 1; --a0)
            for (int a1 = order - 1 - a0; a1 >= 1; --a1) {
                ia[ni][0] = a0;
                ia[ni][1] = a1;
                ia[ni][2] = order - a0 - a1;
                ++ni;
            }
        const int64_t ibase = nv + ke * nedges;
        parallel_for(nc, [&](int64_t c0, int64_t c1) {
            for (int64_t c = c0; c < c1; ++c) {
                const int32_t *cv = mesh->cells + c * 3;
                for (int r = 0; r < ci; ++r) {
                    const int64_t d = ibase + (int64_t)ci * c + r;
                    for (int q = 0; q < dim; ++q)
                        hs.dof_coords[d * dim + q] = ((double)ia[r][0] * mesh->coords[(int64_t)cv[0] * dim + q] +
                                                      (double)ia[r][1] * mesh->coords[(int64_t)cv[1] * dim + q] +
                                                      (double)ia[r][2] * mesh->coords[(int64_t)cv[2] * dim + q]) / order;
                }
            }
        });
    }
    hs.cell_dofs.clear();
    return FEMCG_OK;
}

}  // namespace femcg
