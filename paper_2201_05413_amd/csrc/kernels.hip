// kernels.hip -- gfx950 kernels of the Jacobi-PCG iteration.
//
// One iteration of Jacobi-preconditioned CG (Sect. 2.1's preconditioned
// system with M = diag(A); exit test Eq. (2)) is three bandwidth-bound phases:
//
//   SpMM      q = A p, partial p.q                  -> alpha = rho / p.q
//   update    x += alpha p, r -= alpha q, z = D^-1 r, partial r.z, r.r
//                                                   -> beta, convergence (Eq. 2)
//   p-update  p = D^-1 r + beta p
//
// Every phase is ONE persistent launch over a device table of systems
// (SysTable): the global tile space is the concatenation of every system's
// row tiles, a block walks tiles with an XCD-aware stride (consecutive tiles
// stay on one XCD, so the banded x gather of neighbouring rows hits that XCD's
// L2), and the last tile of a system to finish reduces that system's partial
// dots in a fixed order and writes alpha or beta on the device.  The host
// never sees a scalar inside the iteration.  Reductions are deterministic and
// per system: a system's result does not depend on which other systems share
// the table, nor on the grid size.
//
// Vectors are [n][kp] with the kp right-hand sides of a row contiguous; a row
// is served by kp lanes, so each matrix value and column index is loaded once
// per wavefront row-group and broadcast to its kp lanes (one value load serves
// every right-hand side).  No MFMA: the arithmetic intensity is far below the
// ridge point, the roofline is HBM bandwidth.
#include "internal.h"

namespace femcg {

// ---------------------------------------------------------------------------
// tile scheduling
// ---------------------------------------------------------------------------

__device__ __forceinline__ int find_sys(const SysTable *__restrict__ tab, int64_t t)
{
    int lo = 0, hi = tab->nsys - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (tab->d[mid].tile_base <= t) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// Workgroups are dispatched round-robin over the 8 XCDs (block b on XCD b%8).
// Give XCD x the contiguous tile range [x*T/8, (x+1)*T/8) so that rows close in
// the (banded) matrix are processed on the same L2.
template <typename F>
__device__ __forceinline__ void for_each_tile(int64_t T, F &&f)
{
    const int G = gridDim.x, b = blockIdx.x;
    if (G >= kNumXcd && (G % kNumXcd) == 0) {
        const int xcd = b % kNumXcd, loc = b / kNumXcd, per = G / kNumXcd;
        const int64_t TperX = (T + kNumXcd - 1) / kNumXcd;
        const int64_t base = (int64_t)xcd * TperX;
        for (int64_t j = loc; j < TperX; j += per) {
            const int64_t t = base + j;
            if (t >= T) break;
            f(t);
        }
    } else {
        for (int64_t t = b; t < T; t += G) f(t);
    }
}

// ---------------------------------------------------------------------------
// reductions
// ---------------------------------------------------------------------------

// Lanes l and l' serve the same column iff l = l' (mod kp); sum them.
__device__ __forceinline__ double wave_reduce_cols(double v, int kp)
{
    for (int off = kWave / 2; off >= kp; off >>= 1) v += __shfl_xor(v, off, kWave);
    return v;
}

// dst[i] = sum_{r < rows} src[r*stride + i] for i < W, fixed order: g lanes
// per sum (g | 64), lane `sub` takes rows sub, sub+g, ..., then a fixed xor
// tree over the g lanes.
__device__ __forceinline__ void block_sum_rows(const double *src, int64_t rows, int stride, int W,
                                               double *dst)
{
    int g = kWave;
    while (g > 1 && g * W > kBlock) g >>= 1;
    const int i = threadIdx.x / g, sub = threadIdx.x % g;
    double s = 0.0;
    if (i < W)
        for (int64_t r = sub; r < rows; r += g) s += src[r * stride + i];
    for (int off = g / 2; off >= 1; off >>= 1) s += __shfl_xor(s, off, kWave);
    if (i < W && sub == 0) dst[i] = s;
}

// Commit this tile's per-column partial dots v[0..ndots) and, if this is the
// last tile of its system, reduce every tile of the system into tot[d*kp+j]
// (shared memory) and return true.  Two levels: groups of kGroup tiles, then
// the groups; each level is a fixed-order sum, so the result is independent of
// which block ran which tile.
__device__ bool commit_and_reduce(const SysDesc &D, int64_t tl, int ndots, double *v, double *tot)
{
    __shared__ double red[kBlock / kWave][kDots * kMaxK];
    __shared__ int s_flag;
    const int kp = D.kp, W = ndots * kp, S = kDots * kp;
    const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
    for (int d = 0; d < ndots; ++d) v[d] = wave_reduce_cols(v[d], kp);
    if (lane < kp)
        for (int d = 0; d < ndots; ++d) red[wave][d * kp + lane] = v[d];
    __syncthreads();
    if (threadIdx.x < W) {
        const int i = threadIdx.x;
        D.part[tl * S + i] = ((red[0][i] + red[1][i]) + red[2][i]) + red[3][i];
    }
    __threadfence();
    __syncthreads();
    const int64_t g = tl / kGroup;
    const int64_t ng = (D.ntiles + kGroup - 1) / kGroup;
    const int gcount = (int)min((int64_t)kGroup, (int64_t)D.ntiles - g * kGroup);
    if (threadIdx.x == 0) s_flag = (atomicAdd(&D.gticket[g], 1u) + 1u == (unsigned)gcount);
    __syncthreads();
    if (!s_flag) return false;
    __threadfence();
    if (threadIdx.x == 0) D.gticket[g] = 0u;
    if (ng == 1) {
        block_sum_rows(D.part, gcount, S, W, tot);
        __syncthreads();
        return true;
    }
    block_sum_rows(D.part + g * kGroup * S, gcount, S, W, D.gpart + g * S);
    __threadfence();
    __syncthreads();
    if (threadIdx.x == 0) s_flag = (atomicAdd(&D.st->ticket, 1u) + 1u == (unsigned)ng);
    __syncthreads();
    if (!s_flag) return false;
    __threadfence();
    if (threadIdx.x == 0) D.st->ticket = 0u;
    block_sum_rows(D.gpart, ng, S, W, tot);
    __syncthreads();
    return true;
}

__device__ __forceinline__ void recount_active(SysState *st, int k)
{
    __syncthreads();
    if (threadIdx.x == 0) {
        int n = 0, bad = 0;
        for (int j = 0; j < k; ++j) {
            n += st->active[j];
            bad |= (st->flag[j] == FEMCG_EBREAKDOWN);
        }
        st->n_active = n;
        if (bad) st->status = FEMCG_EBREAKDOWN;
    }
}

// ---------------------------------------------------------------------------
// sparse row product: sum_e A[row][e] * X[col_e][j]
// ---------------------------------------------------------------------------

template <typename T>
__device__ __forceinline__ T row_dot(const SysDesc &D, int64_t row, int j, int kp,
                                     const T *__restrict__ X)
{
    const T *__restrict__ val = (const T *)D.val;
    const int32_t *__restrict__ col = D.col;
    T acc0 = 0, acc1 = 0;
    if (D.format == FEM_FORMAT_SELL) {
        const int sh = D.sell_shift;
        const int64_t C = (int64_t)1 << sh;
        const int64_t base = D.slice_ptr[row >> sh] + (row & (C - 1));
        const int len = D.rowlen[row];
        int e = 0;
        for (; e + 1 < len; e += 2) {
            const int64_t i0 = base + (int64_t)e * C, i1 = i0 + C;
            const int c0 = col[i0], c1 = col[i1];
            const T v0 = val[i0], v1 = val[i1];
            acc0 += v0 * X[(int64_t)c0 * kp + j];
            acc1 += v1 * X[(int64_t)c1 * kp + j];
        }
        if (e < len) {
            const int64_t i0 = base + (int64_t)e * C;
            acc0 += val[i0] * X[(int64_t)col[i0] * kp + j];
        }
    } else {
        const int b = D.rowptr[row], end = D.rowptr[row + 1];
        int t = b;
        for (; t + 1 < end; t += 2) {
            const int c0 = col[t], c1 = col[t + 1];
            const T v0 = val[t], v1 = val[t + 1];
            acc0 += v0 * X[(int64_t)c0 * kp + j];
            acc1 += v1 * X[(int64_t)c1 * kp + j];
        }
        if (t < end) acc0 += val[t] * X[(int64_t)col[t] * kp + j];
    }
    return acc0 + acc1;
}

// ---------------------------------------------------------------------------
// phase 1: q = A p, alpha = rho / p.q
// ---------------------------------------------------------------------------

template <typename T>
__global__ __launch_bounds__(kBlock) void k_spmm(const SysTable *__restrict__ tab, int force)
{
    __shared__ double tot[kDots * kMaxK];
    for_each_tile(tab->total_tiles, [&](int64_t t) {
        const SysDesc D = tab->d[find_sys(tab, t)];
        if (!force && D.st->n_active == 0) return;
        const int64_t tl = t - D.tile_base;
        const int kp = D.kp;
        const int j = threadIdx.x & (kp - 1);
        const int rps = kBlock / kp;
        const int64_t r0 = tl * D.tile_rows, r1 = min(D.n, r0 + D.tile_rows);
        const T *__restrict__ P = (const T *)D.p;
        T *__restrict__ Q = (T *)D.q;
        double v[kDots] = {0.0, 0.0, 0.0};
        for (int64_t row = r0 + threadIdx.x / kp; row < r1; row += rps) {
            const T acc = row_dot<T>(D, row, j, kp, P);
            const int64_t idx = row * kp + j;
            Q[idx] = acc;
            v[0] += (double)P[idx] * (double)acc;
        }
        if (commit_and_reduce(D, tl, 1, v, tot)) {
            SysState *st = D.st;
            if (threadIdx.x < D.k) {
                const int c = threadIdx.x;
                double a = 0.0;
                if (st->active[c]) {
                    const double pq = tot[c];
                    if (!(pq > 0.0) || !isfinite(pq)) {
                        st->active[c] = 0;
                        st->flag[c] = FEMCG_EBREAKDOWN;
                    } else {
                        a = st->rho[c] / pq;
                    }
                }
                st->alpha[c] = a;
            }
            recount_active(st, D.k);
        }
    });
}

// ---------------------------------------------------------------------------
// phase 2: x += alpha p, r -= alpha q, r.z and r.r, then beta / Eq. (2)
// ---------------------------------------------------------------------------

template <typename T>
__global__ __launch_bounds__(kBlock) void k_update(const SysTable *__restrict__ tab, int force)
{
    __shared__ double tot[kDots * kMaxK];
    for_each_tile(tab->total_tiles, [&](int64_t t) {
        const SysDesc D = tab->d[find_sys(tab, t)];
        if (!force && D.st->n_active == 0) return;
        const int64_t tl = t - D.tile_base;
        const int kp = D.kp;
        const int j = threadIdx.x & (kp - 1);
        const int rps = kBlock / kp;
        const int64_t r0 = tl * D.tile_rows, r1 = min(D.n, r0 + D.tile_rows);
        const bool act = j < D.k && (force || D.st->active[j]);
        const double a = act ? D.st->alpha[j] : 0.0;
        T *__restrict__ X = (T *)D.x;
        T *__restrict__ R = (T *)D.r;
        const T *__restrict__ P = (const T *)D.p;
        const T *__restrict__ Q = (const T *)D.q;
        const T *__restrict__ dinv = (const T *)D.dinv;
        double v[kDots] = {0.0, 0.0, 0.0};
        if (act) {
            for (int64_t row = r0 + threadIdx.x / kp; row < r1; row += rps) {
                const int64_t idx = row * kp + j;
                X[idx] = (T)((double)X[idx] + a * (double)P[idx]);
                const T r = (T)((double)R[idx] - a * (double)Q[idx]);
                R[idx] = r;
                const double rd = (double)r;
                v[0] += rd * ((double)dinv[row] * rd);
                v[1] += rd * rd;
            }
        }
        if (commit_and_reduce(D, tl, 2, v, tot)) {
            SysState *st = D.st;
            if (threadIdx.x < D.k) {
                const int c = threadIdx.x;
                if (st->active[c]) {
                    st->iters[c] += 1;
                    const double rz = tot[c], rr = tot[kp + c];
                    st->rr[c] = rr;
                    const double thr = st->tol_rel[c] * st->tol_rel[c] * st->bb[c];
                    if (rr <= thr) {
                        st->active[c] = 0;
                    } else if (!(rz > 0.0) || !isfinite(rz) || !isfinite(rr)) {
                        st->active[c] = 0;
                        st->flag[c] = FEMCG_EBREAKDOWN;
                    } else {
                        st->beta[c] = rz / st->rho[c];
                        st->rho[c] = rz;
                    }
                }
            }
            recount_active(st, D.k);
        }
    });
}

// ---------------------------------------------------------------------------
// phase 3: p = D^-1 r + beta p
// ---------------------------------------------------------------------------

template <typename T>
__global__ __launch_bounds__(kBlock) void k_pupdate(const SysTable *__restrict__ tab, int force)
{
    for_each_tile(tab->total_tiles, [&](int64_t t) {
        const SysDesc D = tab->d[find_sys(tab, t)];
        if (!force && D.st->n_active == 0) return;
        const int64_t tl = t - D.tile_base;
        const int kp = D.kp;
        const int j = threadIdx.x & (kp - 1);
        const int rps = kBlock / kp;
        const int64_t r0 = tl * D.tile_rows, r1 = min(D.n, r0 + D.tile_rows);
        const bool act = j < D.k && (force || D.st->active[j]);
        if (!act) return;
        const double be = D.st->beta[j];
        const T *__restrict__ R = (const T *)D.r;
        T *__restrict__ P = (T *)D.p;
        const T *__restrict__ dinv = (const T *)D.dinv;
        for (int64_t row = r0 + threadIdx.x / kp; row < r1; row += rps) {
            const int64_t idx = row * kp + j;
            P[idx] = (T)((double)dinv[row] * (double)R[idx] + be * (double)P[idx]);
        }
    });
}

// ---------------------------------------------------------------------------
// residual / (re)start: r = b - A x (or r = b, x = 0), p = D^-1 r,
// b.b, r.r, r.z; columns whose Eq. (2) residual exceeds tol become active.
// ---------------------------------------------------------------------------

template <typename T>
__global__ __launch_bounds__(kBlock) void k_residual_init(const SysTable *__restrict__ tab)
{
    __shared__ double tot[kDots * kMaxK];
    for_each_tile(tab->total_tiles, [&](int64_t t) {
        const SysDesc D = tab->d[find_sys(tab, t)];
        const int64_t tl = t - D.tile_base;
        const int kp = D.kp;
        const int j = threadIdx.x & (kp - 1);
        const int rps = kBlock / kp;
        const int64_t r0 = tl * D.tile_rows, r1 = min(D.n, r0 + D.tile_rows);
        T *__restrict__ X = (T *)D.x;
        T *__restrict__ R = (T *)D.r;
        T *__restrict__ P = (T *)D.p;
        const T *__restrict__ B = (const T *)D.b;
        const T *__restrict__ dinv = (const T *)D.dinv;
        const int use_x = D.use_x, write_p = D.write_p;
        double v[kDots] = {0.0, 0.0, 0.0};
        for (int64_t row = r0 + threadIdx.x / kp; row < r1; row += rps) {
            const int64_t idx = row * kp + j;
            const double b = (double)B[idx];
            double ax = 0.0;
            if (use_x) ax = (double)row_dot<T>(D, row, j, kp, X);
            else X[idx] = (T)0;
            const T r = (T)(b - ax);
            R[idx] = r;
            const double rd = (double)r;
            const double z = (double)dinv[row] * rd;
            if (write_p) P[idx] = (T)z;
            v[0] += b * b;
            v[1] += rd * rd;
            v[2] += rd * z;
        }
        if (commit_and_reduce(D, tl, 3, v, tot)) {
            SysState *st = D.st;
            if (threadIdx.x < D.k) {
                const int c = threadIdx.x;
                const double bb = tot[c], rr = tot[kp + c], rz = tot[2 * kp + c];
                st->bb[c] = bb;
                st->rr[c] = rr;
                st->relres[c] = bb > 0.0 ? sqrt(rr / bb) : 0.0;
                int a = 0;
                if (st->flag[c] == 0 && bb > 0.0) {
                    const double thr = st->tol_rel[c] * st->tol_rel[c] * bb;
                    if (!(rr <= thr)) {
                        if (!(rz > 0.0) || !isfinite(rz) || !isfinite(rr)) {
                            st->flag[c] = FEMCG_EBREAKDOWN;
                        } else {
                            a = 1;
                            st->rho[c] = rz;
                        }
                    }
                }
                st->active[c] = a;
            }
            recount_active(st, D.k);
        }
    });
}

// ---------------------------------------------------------------------------
// iterative refinement glue (FP64 outer table, FP32 inner table; the two
// tables describe the same matrices with the same tiling)
// ---------------------------------------------------------------------------

// inner b = r64 / ||r64|| for columns the outer test left active, 0 otherwise;
// inner Eq. (2) threshold max(eta, tol ||b|| / (2 ||r||)).
__global__ __launch_bounds__(kBlock) void k_ir_scale(const SysTable *__restrict__ t64,
                                                     const SysTable *__restrict__ t32)
{
    for_each_tile(t64->total_tiles, [&](int64_t t) {
        const int s = find_sys(t64, t);
        const SysDesc D = t64->d[s];
        const SysDesc E = t32->d[s];
        const int64_t tl = t - D.tile_base;
        const int kp = D.kp;
        const int j = threadIdx.x & (kp - 1);
        const int rps = kBlock / kp;
        const int64_t r0 = tl * D.tile_rows, r1 = min(D.n, r0 + D.tile_rows);
        const bool act = j < D.k && D.st->active[j];
        const double sc = act ? 1.0 / sqrt(D.st->rr[j]) : 0.0;
        const double *__restrict__ R = (const double *)D.r;
        float *__restrict__ Bi = (float *)E.b;
        for (int64_t row = r0 + threadIdx.x / kp; row < r1; row += rps) {
            const int64_t idx = row * kp + j;
            Bi[idx] = act ? (float)(R[idx] * sc) : 0.0f;
        }
        if (tl == 0 && threadIdx.x < D.k) {
            const int c = threadIdx.x;
            SysState *si = E.st;
            const bool a = D.st->active[c];
            si->flag[c] = a ? 0 : 1;
            si->iters[c] = 0;
            const double want = 0.5 * D.st->tol_rel[c] * sqrt(D.st->bb[c] / D.st->rr[c]);
            si->tol_rel[c] = a ? fmax(si->eta, want) : 1.0;
        }
    });
}

// x64 += ||r64|| d32 for columns the outer test left active.
__global__ __launch_bounds__(kBlock) void k_ir_accum(const SysTable *__restrict__ t64,
                                                     const SysTable *__restrict__ t32)
{
    for_each_tile(t64->total_tiles, [&](int64_t t) {
        const int s = find_sys(t64, t);
        const SysDesc D = t64->d[s];
        const SysDesc E = t32->d[s];
        const int64_t tl = t - D.tile_base;
        const int kp = D.kp;
        const int j = threadIdx.x & (kp - 1);
        const int rps = kBlock / kp;
        const int64_t r0 = tl * D.tile_rows, r1 = min(D.n, r0 + D.tile_rows);
        const bool act = j < D.k && D.st->active[j];
        if (!act) return;
        const double sc = sqrt(D.st->rr[j]);
        double *__restrict__ X = (double *)D.x;
        const float *__restrict__ Xi = (const float *)E.x;
        for (int64_t row = r0 + threadIdx.x / kp; row < r1; row += rps) {
            const int64_t idx = row * kp + j;
            X[idx] += sc * (double)Xi[idx];
        }
    });
}

// ---------------------------------------------------------------------------
// layout glue: public [n][k] <-> internal permuted [n][kp]
// ---------------------------------------------------------------------------

__global__ void k_gather(const double *__restrict__ src, int64_t ld, const int32_t *__restrict__ perm,
                         int64_t n, int k, int kp, double *__restrict__ dst)
{
    const int64_t total = n * kp;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = e / kp;
        const int j = (int)(e - i * kp);
        dst[e] = j < k ? src[(int64_t)perm[i] * ld + j] : 0.0;
    }
}

__global__ void k_scatter(const double *__restrict__ src, const int32_t *__restrict__ perm, int64_t n,
                          int k, int kp, const SysState *__restrict__ st, double *__restrict__ dst)
{
    const int64_t total = n * k;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = e / k;
        const int j = (int)(e - i * k);
        const bool zero = st && st->bb[j] == 0.0;
        dst[(int64_t)perm[i] * k + j] = zero ? 0.0 : src[i * kp + j];
    }
}

// B[i][j] = -sum_t K_ID[i][t] gD[col_t][j]  (Dirichlet lifting, zero source)
__global__ void k_lift(const int32_t *__restrict__ rowptr, const int32_t *__restrict__ col,
                       const double *__restrict__ val, const double *__restrict__ gd, int64_t n, int k,
                       double *__restrict__ B)
{
    const int64_t total = n * k;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = e / k;
        const int j = (int)(e - i * k);
        double acc = 0.0;
        for (int t = rowptr[i]; t < rowptr[i + 1]; ++t) acc += val[t] * gd[(int64_t)col[t] * k + j];
        B[e] = -acc;
    }
}

// ---------------------------------------------------------------------------
// host-side launchers
// ---------------------------------------------------------------------------

int grid_for(int64_t total_tiles, int max_grid)
{
    int64_t g = total_tiles < max_grid ? total_tiles : max_grid;
    if (g >= kNumXcd) g -= g % kNumXcd;
    return (int)(g < 1 ? 1 : g);
}

template <typename T>
void launch_phase(int phase, const SysTable *tab, int grid, int force, hipStream_t s)
{
    if (phase == PH_SPMM)
        hipLaunchKernelGGL(k_spmm<T>, dim3(grid), dim3(kBlock), 0, s, tab, force);
    else if (phase == PH_UPDATE)
        hipLaunchKernelGGL(k_update<T>, dim3(grid), dim3(kBlock), 0, s, tab, force);
    else
        hipLaunchKernelGGL(k_pupdate<T>, dim3(grid), dim3(kBlock), 0, s, tab, force);
}

template <typename T>
void launch_residual_init(const SysTable *tab, int grid, hipStream_t s)
{
    hipLaunchKernelGGL(k_residual_init<T>, dim3(grid), dim3(kBlock), 0, s, tab);
}

template void launch_phase<double>(int, const SysTable *, int, int, hipStream_t);
template void launch_phase<float>(int, const SysTable *, int, int, hipStream_t);
template void launch_residual_init<double>(const SysTable *, int, hipStream_t);
template void launch_residual_init<float>(const SysTable *, int, hipStream_t);

static int flat_grid(int64_t total)
{
    int64_t g = (total + kBlock - 1) / kBlock;
    if (g > 4096) g = 4096;
    return (int)(g < 1 ? 1 : g);
}

void launch_gather(const double *src, int64_t ld_src, const int32_t *perm, int64_t n, int k, int kp,
                   double *dst, hipStream_t s)
{
    hipLaunchKernelGGL(k_gather, dim3(flat_grid(n * kp)), dim3(kBlock), 0, s, src, ld_src, perm, n, k,
                       kp, dst);
}

void launch_scatter(const double *src, const int32_t *perm, int64_t n, int k, int kp,
                    const SysState *st, double *dst, hipStream_t s)
{
    hipLaunchKernelGGL(k_scatter, dim3(flat_grid(n * k)), dim3(kBlock), 0, s, src, perm, n, k, kp, st,
                       dst);
}

void launch_lift(const int32_t *rowptr, const int32_t *col, const double *val, const double *gd,
                 int64_t n, int k, double *B, hipStream_t s)
{
    hipLaunchKernelGGL(k_lift, dim3(flat_grid(n * k)), dim3(kBlock), 0, s, rowptr, col, val, gd, n, k,
                       B);
}

void launch_ir_scale(const SysTable *t64, const SysTable *t32, int grid, hipStream_t s)
{
    hipLaunchKernelGGL(k_ir_scale, dim3(grid), dim3(kBlock), 0, s, t64, t32);
}

void launch_ir_accum(const SysTable *t64, const SysTable *t32, int grid, hipStream_t s)
{
    hipLaunchKernelGGL(k_ir_accum, dim3(grid), dim3(kBlock), 0, s, t64, t32);
}

}  // namespace femcg
