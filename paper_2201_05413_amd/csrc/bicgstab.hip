// bicgstab.hip -- BiCGStab right-preconditioned by Block-Jacobi with exact
// blocks, one right-hand side, FP64 (Sect. 3.2: the paper's iterative solver
// is BiCGStab with a Block-Jacobi preconditioner).
//
// Blocks are bs consecutive free DOFs of the public order (the last one may be
// shorter).  Each block's inverse is formed once on the host (Gauss-Jordan
// with partial pivoting) and applied on the device as a dense bs x bs product,
// fused into the kernel that produces the vector it preconditions:
//   K1  rho = (rh, r), ||r||^2 from K5's partials; Eq. (2) test; beta;
//       p = r + beta (p - omega v);  ph = M^-1 p
//   K2  v = A ph;  partial (rh, v)
//   K3  alpha = rho / (rh, v);  s = r - alpha v;  sh = M^-1 s;  partial (s, s)
//   K4  unless ||s|| <= tol ||b||:  t = A sh;  partials (t, s), (t, t)
//   K5  omega = (t, s) / (t, t);  x += alpha ph + omega sh;  r = s - omega t
//       (x += alpha ph and r = s when ||s|| <= tol ||b||: the solve then
//       stops);  partials (rh, r), (r, r)
// A Lanczos near-breakdown, |rho| <= 1e-14 ||rh|| ||r||, restarts the
// iteration from x with rh = r (at most 100 times): with zero source the
// lifted b, hence the first rh, lives on the rows next to the boundary only,
// and rho can decay far faster than r there.
// Every block of a kernel reduces the partials it needs in one fixed order,
// so all blocks derive the same scalars; block 0 records alpha, rho and
// omega in the state for the kernels that follow.  No kernel reads a partial
// slot it writes, and the state fields a kernel writes are read only by later
// kernels (a block that sees another block's "done" in the same kernel would
// have taken the same decision itself).
//
// An optional row scale D (positive, per row) turns the system into
// D A x = D b, the form A = B^-1 L of Sect. 2.2 when D is the inverse lumped
// mass: b is scaled where it is gathered, every product row is scaled as it
// is produced, and the block inverses are those of the scaled rows.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <exception>
#include <memory>
#include <new>
#include <vector>

#include "engine.h"

namespace femcg {

namespace {

constexpr int kB = 256;          // threads per block
constexpr int kGridMax = 1024;   // blocks, i.e. partials per dot
constexpr int kRowLoads = 8;     // entries per batch of a row product (even)
enum { SL_B = 0, SL_C = 1, SL_D = 2, SL_E = 3, SL_X = 4, kSlots = 5 };

struct BcgState {
    double rho_old, alpha, omega, bb, tol2;
    double rr;      // ||r||^2 seen by the last K1
    double rhrh;    // ||rh||^2 of this start
    double bad;     // the scalar that broke down
    long long iters, max_iter;
    int done;       // 0 running, 1 converged, 2 iteration cap, 3 Lanczos restart,
                    // -1 / -2 / -3 breakdown in rho / (rh, v) / omega
    int stop_next;  // K5 stopped at s: K1 ends the solve
};

struct BcgArgs {
    int64_t n;
    int format, sell_shift;
    const int32_t *rowptr;
    const int64_t *slice_ptr;
    const int32_t *rowlen;
    const int32_t *col;
    const double *val;
    int bs;
    const double *binv;     // [nb][bs][bs]
    const int32_t *iperm;   // public free row -> internal row
    const double *dsc;      // row scale, internal order, or nullptr
    double *b, *x, *r, *rh, *p, *ph, *v, *s, *sh, *t;
    double *part;           // [kSlots][grid][2]
    BcgState *st;
};

// Entries alternate between two sums (even and odd positions of the row,
// each in order).  A batch loads kRowLoads indices and values at once, then
// their gathers: entries past the row's end take its last index and a zero
// value, so every load is in bounds and none waits on a branch.
__device__ __forceinline__ double row_dot(const BcgArgs &a, int64_t row, const double *__restrict__ x)
{
    double acc0 = 0.0, acc1 = 0.0;
    int64_t base, stride;
    int len;
    if (a.format == FEM_FORMAT_SELL) {
        stride = (int64_t)1 << a.sell_shift;
        base = a.slice_ptr[row >> a.sell_shift] + (row & (stride - 1));
        len = a.rowlen[row];
    } else {
        stride = 1;
        base = a.rowptr[row];
        len = a.rowptr[row + 1] - (int32_t)base;
    }
    for (int e = 0; e < len; e += kRowLoads) {
        int32_t c[kRowLoads];
        double v[kRowLoads], xv[kRowLoads];
#pragma unroll
        for (int u = 0; u < kRowLoads; ++u) {
            const int64_t i = base + (int64_t)min(e + u, len - 1) * stride;
            c[u] = a.col[i];
            v[u] = a.val[i] * (e + u < len ? 1.0 : 0.0);  // a factor, not a select (no branch round the load)
        }
#pragma unroll
        for (int u = 0; u < kRowLoads; ++u) xv[u] = x[c[u]];
#pragma unroll
        for (int u = 0; u < kRowLoads; u += 2) {
            acc0 += v[u] * xv[u];
            acc1 += v[u + 1] * xv[u + 1];
        }
    }
    return acc0 + acc1;
}

// The rows a thread visits in a product kernel.  Blocks are dispatched to the
// XCDs round-robin (block b on XCD b mod kNumXcd), so each XCD takes one
// contiguous share of the rows and its blocks walk that share in kB-row
// chunks: rows that gather the same neighbours meet in one L2.  Grids that are
// not a multiple of the XCD count use the plain grid stride.
struct RowWalk {
    int64_t begin, end, step;
};
__device__ __forceinline__ RowWalk row_walk(int64_t n)
{
    const int G = gridDim.x;
    if (G % kNumXcd != 0) return {(int64_t)blockIdx.x * kB + threadIdx.x, n, (int64_t)G * kB};
    const int x = blockIdx.x % kNumXcd, j = blockIdx.x / kNumXcd;
    const int64_t share = (n + kNumXcd - 1) / kNumXcd;
    const int64_t lo = min<int64_t>(n, x * share), hi = min<int64_t>(n, lo + share);
    return {lo + (int64_t)j * kB + threadIdx.x, hi, (int64_t)(G / kNumXcd) * kB};
}

// row of the (possibly row-scaled) operator
__device__ __forceinline__ double op_row(const BcgArgs &a, int64_t row, const double *__restrict__ x)
{
    const double y = row_dot(a, row, x);
    return a.dsc ? a.dsc[row] * y : y;
}

// block sums of v[0..1] in a fixed tree, stored as this block's partials
__device__ void write_partials(const BcgArgs &a, int slot, double v0, double v1)
{
    __shared__ double red[2][kB];
    red[0][threadIdx.x] = v0;
    red[1][threadIdx.x] = v1;
    __syncthreads();
    for (int off = kB / 2; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) {
            red[0][threadIdx.x] += red[0][threadIdx.x + off];
            red[1][threadIdx.x] += red[1][threadIdx.x + off];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        double *dst = a.part + ((int64_t)slot * gridDim.x + blockIdx.x) * 2;
        dst[0] = red[0][0];
        dst[1] = red[1][0];
    }
}

// the two sums of one partial slot, in the same order in every block
__device__ void reduce_slot(const BcgArgs &a, int slot, double out[2])
{
    __shared__ double red[2][kB];
    const int G = gridDim.x;
    const double *src = a.part + (int64_t)slot * G * 2;
    double s0 = 0.0, s1 = 0.0;
    for (int g = threadIdx.x; g < G; g += kB) {
        s0 += src[2 * g];
        s1 += src[2 * g + 1];
    }
    red[0][threadIdx.x] = s0;
    red[1][threadIdx.x] = s1;
    __syncthreads();
    for (int off = kB / 2; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) {
            red[0][threadIdx.x] += red[0][threadIdx.x + off];
            red[1][threadIdx.x] += red[1][threadIdx.x + off];
        }
        __syncthreads();
    }
    out[0] = red[0][0];
    out[1] = red[1][0];
    __syncthreads();
}

// the sums of two partial slots in one pass, each in reduce_slot's order
// (so the results are those of two reduce_slot calls)
__device__ void reduce_two_slots(const BcgArgs &a, int s0, int s1, double o0[2], double o1[2])
{
    __shared__ double red[4][kB];
    const int G = gridDim.x;
    const double *p0 = a.part + (int64_t)s0 * G * 2, *p1 = a.part + (int64_t)s1 * G * 2;
    double v[4] = {0.0, 0.0, 0.0, 0.0};
    for (int g = threadIdx.x; g < G; g += kB) {
        v[0] += p0[2 * g];
        v[1] += p0[2 * g + 1];
        v[2] += p1[2 * g];
        v[3] += p1[2 * g + 1];
    }
#pragma unroll
    for (int c = 0; c < 4; ++c) red[c][threadIdx.x] = v[c];
    __syncthreads();
    for (int off = kB / 2; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) {
#pragma unroll
            for (int c = 0; c < 4; ++c) red[c][threadIdx.x] += red[c][threadIdx.x + off];
        }
        __syncthreads();
    }
    o0[0] = red[0][0];
    o0[1] = red[1][0];
    o1[0] = red[2][0];
    o1[1] = red[3][0];
    __syncthreads();
}

// For every public free row i: w = f(internal row) is stored to out1, and
// out2 = M^-1 w for the row's block.  A sub-pass of a workgroup covers whole
// blocks (kB / bs of them), staged in LDS; each thread keeps kU sub-passes in
// flight, all loads issued before any store (out1 may be one of f's inputs,
// at the same index only).  Blocks of one row need no staging and no public
// order: those run over internal rows, with the inverse diagonal kept in
// internal order.  Returns this thread's sum of w^2.
constexpr int kU = 4;

template <typename F>
__device__ double block_apply(const BcgArgs &a, F &&f, double *__restrict__ out1, double *__restrict__ out2)
{
    __shared__ double sw[kU][kB];
    const int bs = a.bs;
    double w2 = 0.0;
    if (bs == 1) {
        const int64_t stride = (int64_t)gridDim.x * kB;
        for (int64_t i0 = (int64_t)blockIdx.x * kB + threadIdx.x; i0 < a.n; i0 += kU * stride) {
            double w[kU];
#pragma unroll
            for (int u = 0; u < kU; ++u) {
                const int64_t i = i0 + u * stride;
                w[u] = i < a.n ? f((int32_t)i) : 0.0;
            }
#pragma unroll
            for (int u = 0; u < kU; ++u) {
                const int64_t i = i0 + u * stride;
                if (i < a.n) {
                    out1[i] = w[u];
                    out2[i] = a.binv[i] * w[u];
                    w2 += w[u] * w[u];
                }
            }
        }
        return w2;
    }
    const int R = (kB / bs) * bs;
    const int lr = threadIdx.x, q = lr % bs;
    const int64_t npass = (a.n + (int64_t)kU * R - 1) / ((int64_t)kU * R);
    for (int64_t c = blockIdx.x; c < npass; c += gridDim.x) {
        int32_t ii[kU];
        double w[kU];
#pragma unroll
        for (int u = 0; u < kU; ++u) {
            const int64_t i = (c * kU + u) * R + lr;
            ii[u] = (lr < R && i < a.n) ? a.iperm[i] : -1;
        }
#pragma unroll
        for (int u = 0; u < kU; ++u) w[u] = ii[u] >= 0 ? f(ii[u]) : 0.0;
#pragma unroll
        for (int u = 0; u < kU; ++u) {
            if (ii[u] >= 0) {
                out1[ii[u]] = w[u];
                w2 += w[u] * w[u];
            }
            sw[u][lr] = w[u];
        }
        __syncthreads();
#pragma unroll
        for (int u = 0; u < kU; ++u) {
            if (ii[u] >= 0) {
                const int64_t i0 = (c * kU + u) * R + lr - q;
                const int m = (int)min<int64_t>(bs, a.n - i0);
                const double *Bi = a.binv + ((i0 / bs) * bs + q) * (int64_t)bs;
                double z = 0.0;
                for (int j = 0; j < m; ++j) z += Bi[j] * sw[u][lr - q + j];
                out2[ii[u]] = z;
            }
        }
        __syncthreads();
    }
    return w2;
}

__device__ __forceinline__ bool lead() { return blockIdx.x == 0 && threadIdx.x == 0; }

// (b, b) into slot X
__global__ __launch_bounds__(kB) void k_bcg_bb(BcgArgs a)
{
    double acc = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * kB + threadIdx.x; i < a.n; i += (int64_t)gridDim.x * kB) acc += a.b[i] * a.b[i];
    write_partials(a, SL_X, acc, 0.0);
}

// start (or restart from x): r = b - A x (x = 0: r = b), rh = r, p = v = 0;
// partials (rh, r), (r, r) into slot E
__global__ __launch_bounds__(kB) void k_bcg_init(BcgArgs a, int use_x)
{
    double acc = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * kB + threadIdx.x; i < a.n; i += (int64_t)gridDim.x * kB) {
        double r;
        if (use_x) {
            r = a.b[i] - op_row(a, i, a.x);
        } else {
            r = a.b[i];
            a.x[i] = 0.0;
        }
        a.r[i] = r;
        a.rh[i] = r;
        a.p[i] = 0.0;
        a.v[i] = 0.0;
        acc += r * r;
    }
    write_partials(a, SL_E, acc, acc);
}

// K1
__global__ __launch_bounds__(kB) void k_bcg_p(BcgArgs a)
{
    BcgState *st = a.st;
    if (st->done) return;
    double e[2];
    reduce_slot(a, SL_E, e);
    const double rho = e[0], rr = e[1];
    if (lead()) st->rr = rr;
    if (st->stop_next || rr <= st->tol2 * st->bb) {
        if (lead()) st->done = 1;
        return;
    }
    if (st->iters >= st->max_iter) {
        if (lead()) st->done = 2;
        return;
    }
    if (!isfinite(rho)) {
        if (lead()) {
            st->bad = rho;
            st->done = -1;
        }
        return;
    }
    if (!(fabs(rho) > 1e-14 * sqrt(st->rhrh) * sqrt(rr))) {
        if (lead()) {
            st->bad = rho;
            st->done = 3;
        }
        return;
    }
    const double beta = (rho / st->rho_old) * (st->alpha / st->omega);
    const double omega = st->omega;
    block_apply(
        a, [&](int32_t ii) { return a.r[ii] + beta * (a.p[ii] - omega * a.v[ii]); }, a.p, a.ph);
}

// K2
__global__ __launch_bounds__(kB) void k_bcg_v(BcgArgs a)
{
    if (a.st->done) return;
    double acc = 0.0;
    const RowWalk w = row_walk(a.n);
    for (int64_t i = w.begin; i < w.end; i += w.step) {
        const double v = op_row(a, i, a.ph);
        a.v[i] = v;
        acc += a.rh[i] * v;
    }
    write_partials(a, SL_B, acc, 0.0);
}

// K3
__global__ __launch_bounds__(kB) void k_bcg_s(BcgArgs a)
{
    BcgState *st = a.st;
    if (st->done) return;
    double e[2], bsum[2];
    reduce_two_slots(a, SL_E, SL_B, e, bsum);
    const double rho = e[0], sig = bsum[0];
    if (sig == 0.0 || !isfinite(sig)) {
        if (lead()) {
            st->bad = sig;
            st->done = -2;
        }
        return;
    }
    const double alpha = rho / sig;
    const double w2 = block_apply(
        a, [&](int32_t ii) { return a.r[ii] - alpha * a.v[ii]; }, a.s, a.sh);
    write_partials(a, SL_C, w2, 0.0);
    if (lead()) {
        st->alpha = alpha;
        st->rho_old = rho;
        st->iters += 1;
    }
}

// K4
__global__ __launch_bounds__(kB) void k_bcg_t(BcgArgs a)
{
    BcgState *st = a.st;
    if (st->done) return;
    double c[2];
    reduce_slot(a, SL_C, c);
    if (c[0] <= st->tol2 * st->bb) return;  // stops at s: t is not needed
    double ts = 0.0, tt = 0.0;
    const RowWalk w = row_walk(a.n);
    for (int64_t i = w.begin; i < w.end; i += w.step) {
        const double t = op_row(a, i, a.sh);
        a.t[i] = t;
        ts += t * a.s[i];
        tt += t * t;
    }
    write_partials(a, SL_D, ts, tt);
}

// K5
__global__ __launch_bounds__(kB) void k_bcg_xr(BcgArgs a)
{
    BcgState *st = a.st;
    if (st->done) return;
    double c[2], d[2];
    reduce_two_slots(a, SL_C, SL_D, c, d);  // D is stale (and unused) at a half step
    const double alpha = st->alpha;
    const bool half = c[0] <= st->tol2 * st->bb;
    double omega = 0.0;
    if (!half) {
        omega = d[0] / d[1];
        if (omega == 0.0 || !isfinite(omega)) {
            if (lead()) {
                st->bad = omega;
                st->done = -3;
            }
            return;
        }
    }
    double rhr = 0.0, rr = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * kB + threadIdx.x; i < a.n; i += (int64_t)gridDim.x * kB) {
        double r;
        if (half) {
            a.x[i] += alpha * a.ph[i];
            r = a.s[i];
        } else {
            a.x[i] += alpha * a.ph[i] + omega * a.sh[i];
            r = a.s[i] - omega * a.t[i];
        }
        a.r[i] = r;
        rhr += a.rh[i] * r;
        rr += r * r;
    }
    write_partials(a, SL_E, rhr, rr);
    if (lead()) {
        if (half) st->stop_next = 1;
        else st->omega = omega;
    }
}

// true residual ||b - A x||^2 into slot X
__global__ __launch_bounds__(kB) void k_bcg_true(BcgArgs a)
{
    double acc = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * kB + threadIdx.x; i < a.n; i += (int64_t)gridDim.x * kB) {
        const double d = a.b[i] - op_row(a, i, a.x);
        acc += d * d;
    }
    write_partials(a, SL_X, acc, 0.0);
}

// public <-> internal order (the right-hand side scaled by the row scale)
__global__ void k_bcg_gather(const double *__restrict__ B, const int32_t *__restrict__ iperm,
                             const double *__restrict__ dsc, int64_t n, double *__restrict__ b)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int32_t ii = iperm[i];
        b[ii] = dsc ? dsc[ii] * B[i] : B[i];
    }
}
__global__ void k_bcg_scatter(const double *__restrict__ x, const int32_t *__restrict__ iperm, int64_t n,
                              double *__restrict__ X)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        X[i] = x[iperm[i]];
}

#define BCHK(call)                                                                            \
    do {                                                                                      \
        hipError_t e_ = (call);                                                               \
        if (e_ != hipSuccess) return fail(FEMCG_EDEVICE, "%s: %s", #call, hipGetErrorString(e_)); \
    } while (0)

// Inverse of each diagonal block of D A (public order; D = diag(scale), or
// the identity when scale is empty) by Gauss-Jordan elimination with partial
// pivoting; returns false for a singular block.
bool block_inverses(const HostSystem &hs, int bs, const std::vector<double> &scale, std::vector<double> &inv)
{
    const int64_t n = hs.nfree, nb = (n + bs - 1) / bs;
    inv.assign((size_t)nb * bs * bs, 0.0);
    std::atomic<int> nbad{0};
    parallel_for(nb, [&](int64_t b0, int64_t b1) {
        std::vector<double> M((size_t)bs * 2 * bs);
        for (int64_t b = b0; b < b1; ++b) {
            const int64_t r0 = b * bs;
            const int m = (int)std::min<int64_t>(bs, n - r0);
            std::fill(M.begin(), M.end(), 0.0);
            for (int i = 0; i < m; ++i) {
                const double di = scale.empty() ? 1.0 : scale[r0 + i];
                for (int64_t e = hs.a_rowptr[r0 + i]; e < hs.a_rowptr[r0 + i + 1]; ++e) {
                    const int64_t c = hs.a_col[e];
                    if (c >= r0 && c < r0 + m) M[(size_t)i * 2 * bs + (c - r0)] += di * hs.a_val[e];
                }
                M[(size_t)i * 2 * bs + bs + i] = 1.0;
            }
            bool ok = true;
            for (int c = 0; c < m && ok; ++c) {
                int piv = c;
                for (int r = c + 1; r < m; ++r)
                    if (std::fabs(M[(size_t)r * 2 * bs + c]) > std::fabs(M[(size_t)piv * 2 * bs + c])) piv = r;
                if (M[(size_t)piv * 2 * bs + c] == 0.0) {
                    ok = false;
                    break;
                }
                if (piv != c)
                    for (int j = 0; j < 2 * bs; ++j) std::swap(M[(size_t)c * 2 * bs + j], M[(size_t)piv * 2 * bs + j]);
                const double d = M[(size_t)c * 2 * bs + c];
                for (int j = 0; j < 2 * bs; ++j) M[(size_t)c * 2 * bs + j] /= d;
                for (int r = 0; r < m; ++r)
                    if (r != c) {
                        const double f = M[(size_t)r * 2 * bs + c];
                        if (f != 0.0)
                            for (int j = 0; j < 2 * bs; ++j) M[(size_t)r * 2 * bs + j] -= f * M[(size_t)c * 2 * bs + j];
                    }
            }
            if (!ok) {
                nbad.fetch_add(1);
                continue;
            }
            for (int i = 0; i < m; ++i)
                for (int j = 0; j < m; ++j) inv[((size_t)b * bs + i) * bs + j] = M[(size_t)i * 2 * bs + bs + j];
        }
    });
    return nbad.load() == 0;
}

int bcg_prepare(fem_matrix *A, int bs, const double *row_scale)
{
    const int64_t n = A->sc.n;
    if (A->bcg && A->bcg->bs == bs) {
        const std::vector<double> &sc = A->bcg->scale;
        const bool same = row_scale ? (!sc.empty() && std::memcmp(sc.data(), row_scale, sizeof(double) * n) == 0)
                                    : sc.empty();
        if (same) return FEMCG_OK;
    }
    const double t0 = now_s();
    A->bcg.reset();
    auto W = std::make_unique<BcgWork>();
    if (row_scale) W->scale.assign(row_scale, row_scale + n);
    W->bs = bs;
    W->n = n;
    W->nb = (n + bs - 1) / bs;
    W->grid = (int)std::max<int64_t>(1, std::min<int64_t>(kGridMax, (n + kB - 1) / kB));
    std::vector<double> inv;
    if (!block_inverses(A->hs, bs, W->scale, inv)) return fail(FEMCG_EBREAKDOWN, "singular diagonal block (block size %d)", bs);
    std::vector<int32_t> iperm(n);
    for (int64_t i = 0; i < n; ++i) iperm[A->sc.perm[i]] = (int32_t)i;
    if (bs == 1) {  // one-row blocks are applied in internal order
        std::vector<double> d(n);
        for (int64_t i = 0; i < n; ++i) d[iperm[i]] = inv[i];
        inv.swap(d);
    }
    auto al = [](size_t b) { return (b + 255) & ~(size_t)255; };
    const size_t vb = al(sizeof(double) * std::max<int64_t>(n, 1));
    const size_t ib = al(sizeof(double) * inv.size()), pb = al(sizeof(int32_t) * std::max<int64_t>(n, 1));
    const size_t partb = al(sizeof(double) * kSlots * W->grid * 2), stb = al(sizeof(BcgState));
    const size_t db = W->scale.empty() ? 0 : vb;
    W->bytes = ib + pb + db + 10 * vb + partb + stb;
    if (hipMalloc((void **)&W->mem, W->bytes) != hipSuccess) {
        W->mem = nullptr;
        return fail(FEMCG_ENOMEM, "BiCGStab workspace (%zu bytes)", W->bytes);
    }
    char *q = W->mem;
    W->binv = (double *)q;
    q += ib;
    W->iperm = (int32_t *)q;
    q += pb;
    if (db) {
        W->dsc = (double *)q;
        q += db;
    }
    double **vecs[10] = {&W->b, &W->x, &W->r, &W->rh, &W->p, &W->ph, &W->v, &W->s, &W->sh, &W->t};
    for (auto v : vecs) {
        *v = (double *)q;
        q += vb;
    }
    W->part = (double *)q;
    q += partb;
    W->st = q;
    if (hipHostMalloc(&W->h_st, sizeof(BcgState), hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc((void **)&W->h_part, sizeof(double) * W->grid * 2, hipHostMallocDefault) != hipSuccess)
        return fail(FEMCG_ENOMEM, "pinned host buffers");
    BCHK(hipMemcpy(W->binv, inv.data(), sizeof(double) * inv.size(), hipMemcpyHostToDevice));
    BCHK(hipMemcpy(W->iperm, iperm.data(), sizeof(int32_t) * n, hipMemcpyHostToDevice));
    if (db) {
        std::vector<double> dint(n);
        for (int64_t i = 0; i < n; ++i) dint[iperm[i]] = W->scale[i];
        BCHK(hipMemcpy(W->dsc, dint.data(), sizeof(double) * n, hipMemcpyHostToDevice));
    }
    W->setup_s = now_s() - t0;
    A->bcg = std::move(W);
    return FEMCG_OK;
}

BcgArgs bcg_args(const fem_matrix *A)
{
    const BcgWork *W = A->bcg.get();
    const DevSparse &d = A->dev;
    BcgArgs a{};
    a.n = W->n;
    a.format = d.format;
    int sh = 0;
    while ((1 << sh) < d.C) ++sh;
    a.sell_shift = sh;
    a.rowptr = d.rowptr;
    a.slice_ptr = d.slice_ptr;
    a.rowlen = d.rowlen;
    a.col = d.col;
    a.val = (const double *)d.val64;
    a.bs = W->bs;
    a.binv = W->binv;
    a.iperm = W->iperm;
    a.dsc = W->dsc;
    a.b = W->b;
    a.x = W->x;
    a.r = W->r;
    a.rh = W->rh;
    a.p = W->p;
    a.ph = W->ph;
    a.v = W->v;
    a.s = W->s;
    a.sh = W->sh;
    a.t = W->t;
    a.part = W->part;
    a.st = (BcgState *)W->st;
    return a;
}

// one poll window: m iterations of the five phase kernels
void enqueue_window(const BcgArgs &a, int G, int m, hipStream_t s)
{
    for (int i = 0; i < m; ++i) {
        hipLaunchKernelGGL(k_bcg_p, dim3(G), dim3(kB), 0, s, a);
        hipLaunchKernelGGL(k_bcg_v, dim3(G), dim3(kB), 0, s, a);
        hipLaunchKernelGGL(k_bcg_s, dim3(G), dim3(kB), 0, s, a);
        hipLaunchKernelGGL(k_bcg_t, dim3(G), dim3(kB), 0, s, a);
        hipLaunchKernelGGL(k_bcg_xr, dim3(G), dim3(kB), 0, s, a);
    }
}

// The window captured once per workspace (its arguments are fixed: the
// workspace is rebuilt when the format, the block size or the row scale
// changes) on a private stream, replayed on the caller's stream.
int ensure_window_graph(BcgWork *W, const BcgArgs &a, int m)
{
    if (W->gexec) return FEMCG_OK;
    if (!W->cap) {
        hipStream_t cs = nullptr;
        BCHK(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
        W->cap = cs;
    }
    hipStream_t cs = (hipStream_t)W->cap;
    hipGraph_t g = nullptr;
    BCHK(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
    enqueue_window(a, W->grid, m, cs);
    const hipError_t le = hipGetLastError();
    const hipError_t ce = hipStreamEndCapture(cs, &g);
    if (le != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return fail(FEMCG_EDEVICE, "BiCGStab graph capture: %s", hipGetErrorString(le));
    }
    if (ce != hipSuccess) return fail(FEMCG_EDEVICE, "BiCGStab graph capture: %s", hipGetErrorString(ce));
    hipGraphExec_t ge = nullptr;
    const hipError_t ie = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (ie != hipSuccess) return fail(FEMCG_EDEVICE, "BiCGStab graph instantiate: %s", hipGetErrorString(ie));
    W->gexec = ge;
    return FEMCG_OK;
}

// sum of value `comp` of the grid's partials of a slot, in block order
int read_slot(BcgWork *W, hipStream_t s, int slot, int comp, double *out)
{
    BCHK(hipMemcpyAsync(W->h_part, W->part + (size_t)slot * W->grid * 2, sizeof(double) * W->grid * 2,
                        hipMemcpyDeviceToHost, s));
    BCHK(hipStreamSynchronize(s));
    double acc = 0.0;
    for (int g = 0; g < W->grid; ++g) acc += W->h_part[2 * g + comp];
    *out = acc;
    return FEMCG_OK;
}

}  // namespace

BcgWork::~BcgWork()
{
    if (gexec) (void)hipGraphExecDestroy((hipGraphExec_t)gexec);
    if (cap) (void)hipStreamDestroy((hipStream_t)cap);
    if (mem) (void)hipFree(mem);
    if (h_st) (void)hipHostFree(h_st);
    if (h_part) (void)hipHostFree(h_part);
}

}  // namespace femcg

using namespace femcg;

extern "C" {

static int bicgstab_solve_impl(fem_matrix *A, const double *B, double *X, double tol, int32_t block_size,
                               const double *row_scale, int64_t max_iter, void *stream, bicgstab_stats_t *stats)
{
    if (!A || !B || !X) return fail(FEMCG_EINVAL, "NULL argument");
    if (int rc = require_device(A)) return rc;
    if (!(tol > 0.0) || !std::isfinite(tol)) return fail(FEMCG_EINVAL, "tol must be positive and finite");
    if (block_size < 1 || block_size > 64) return fail(FEMCG_EINVAL, "block_size must be 1..64");
    if (max_iter < 0) return fail(FEMCG_EINVAL, "max_iter must be >= 0");
    if (row_scale)
        for (int64_t i = 0; i < A->sc.n; ++i)
            if (!(row_scale[i] > 0.0) || !std::isfinite(row_scale[i]))
                return fail(FEMCG_EINVAL, "row_scale[%lld] = %g: entries must be finite and > 0", (long long)i,
                            row_scale[i]);
    const double t_begin = now_s();
    int rc = bcg_prepare(A, block_size, row_scale);
    if (rc) return rc;
    BcgWork *W = A->bcg.get();
    hipStream_t s = (hipStream_t)stream;
    const int64_t n = W->n;
    const int G = W->grid;
    const BcgArgs a = bcg_args(A);
    const int ge = (int)std::min<int64_t>(4096, (n + 255) / 256 + 1);
    hipLaunchKernelGGL(k_bcg_gather, dim3(ge), dim3(256), 0, s, B, W->iperm, (const double *)W->dsc, n, W->b);
    hipLaunchKernelGGL(k_bcg_bb, dim3(G), dim3(kB), 0, s, a);
    BCHK(hipGetLastError());
    double bb = 0.0;
    if ((rc = read_slot(W, s, SL_X, 0, &bb))) return rc;
    if (!std::isfinite(bb)) return fail(FEMCG_EBREAKDOWN, "non-finite right-hand side");
    BcgState *hst = (BcgState *)W->h_st;
    const int64_t cap = max_iter > 0 ? max_iter : default_max_iter(n);
    int64_t iters = 0;
    int restarts = 0, soft = 0, status = FEMCG_OK;
    double rel = 0.0;
    if (bb == 0.0) {
        BCHK(hipMemsetAsync(X, 0, sizeof(double) * n, s));
        BCHK(hipStreamSynchronize(s));
    } else {
        const int m = 32;  // iterations enqueued between polls
        const char *gv = std::getenv("FEMCG_BCG_GRAPH");
        const bool use_graph = !(gv && gv[0] == '0');
        if (use_graph && (rc = ensure_window_graph(W, a, m))) return rc;
        int use_x = 0;
        for (;;) {
            hipLaunchKernelGGL(k_bcg_init, dim3(G), dim3(kB), 0, s, a, use_x);
            BCHK(hipGetLastError());
            double rhrh = 0.0;
            if ((rc = read_slot(W, s, SL_E, 1, &rhrh))) return rc;
            BcgState init{};
            init.rho_old = init.alpha = init.omega = 1.0;
            init.bb = bb;
            init.tol2 = tol * tol;
            init.rhrh = rhrh;
            init.iters = iters;
            init.max_iter = cap;
            std::memcpy(hst, &init, sizeof(init));
            BCHK(hipMemcpyAsync(W->st, hst, sizeof(BcgState), hipMemcpyHostToDevice, s));
            for (;;) {
                if (use_graph) BCHK(hipGraphLaunch((hipGraphExec_t)W->gexec, s));
                else enqueue_window(a, G, m, s);
                BCHK(hipGetLastError());
                BCHK(hipMemcpyAsync(hst, W->st, sizeof(BcgState), hipMemcpyDeviceToHost, s));
                BCHK(hipStreamSynchronize(s));
                if (hst->done) break;
                if (std::getenv("FEMCG_BCG_TRACE") && hst->iters % 512 < 32)
                    fprintf(stderr, "bicgstab: %lld iterations, ||r|| / ||b|| = %.3e\n", (long long)hst->iters,
                            std::sqrt(hst->rr / bb));
            }
            iters = hst->iters;
            if (hst->done == 3) {  // Lanczos near-breakdown: restart from x
                if (soft < 100 && iters < cap) {
                    ++soft;
                    use_x = 1;
                    continue;
                }
                status = fail(FEMCG_EBREAKDOWN, "BiCGStab: %d Lanczos restarts without convergence (%lld iterations)",
                              soft, (long long)iters);
                break;
            }
            if (hst->done < 0) {
                static const char *what[] = {"rho = (rh, r)", "(rh, v)", "omega"};
                status = fail(FEMCG_EBREAKDOWN, "BiCGStab breakdown after %lld iterations: %s = %g (||r|| / ||b|| = %g)",
                              (long long)iters, what[std::min(2, -hst->done - 1)], hst->bad, std::sqrt(hst->rr / bb));
                break;
            }
            if (std::getenv("FEMCG_BCG_TRACE"))
                fprintf(stderr, "bicgstab: %lld iterations, ||r|| / ||b|| = %.3e\n", (long long)hst->iters,
                        std::sqrt(hst->rr / bb));
            hipLaunchKernelGGL(k_bcg_true, dim3(G), dim3(kB), 0, s, a);
            BCHK(hipGetLastError());
            double rr = 0.0;
            if ((rc = read_slot(W, s, SL_X, 0, &rr))) return rc;
            rel = std::sqrt(rr / bb);
            if (hst->done == 2) {
                status = rel <= tol ? FEMCG_OK : FEMCG_WARN_MAXITER;
                break;
            }
            if (rel <= tol) break;
            if (restarts >= 3) {  // the true residual still misses Eq. (2)
                status = FEMCG_WARN_MAXITER;
                break;
            }
            ++restarts;
            use_x = 1;
        }
        hipLaunchKernelGGL(k_bcg_scatter, dim3(ge), dim3(256), 0, s, W->x, W->iperm, n, X);
        BCHK(hipGetLastError());
        BCHK(hipStreamSynchronize(s));
    }
    if (stats) {
        std::memset(stats, 0, sizeof(*stats));
        stats->iters = iters;
        stats->relres = rel;
        stats->restarts = restarts + soft;
        stats->block_size = block_size;
        stats->nblocks = W->nb;
        stats->setup_s = W->setup_s;
        stats->solve_s = now_s() - t_begin;
        // per iteration: two matrix passes, two block-inverse and row-map
        // passes, and 23 vector passes (K1 5, K2 3, K3 4, K4 3, K5 8), plus
        // the row scale read by each matrix pass
        const double nnz = (double)A->sc.stored;
        const double per = 2.0 * (nnz * 12.0 + 4.0 * (n + 1)) + 2.0 * (8.0 * n * block_size + 4.0 * n) +
                           (23.0 + (W->dsc ? 2.0 : 0.0)) * 8.0 * n;
        stats->bytes = per * (double)iters;
    }
    return status;
}

int bicgstab_solve(fem_matrix *A, const double *B, double *X, double tol, int32_t block_size,
                   const double *row_scale, int64_t max_iter, void *stream, bicgstab_stats_t *stats)
{
    try {
        return bicgstab_solve_impl(A, B, X, tol, block_size, row_scale, max_iter, stream, stats);
    } catch (const std::bad_alloc &) {
        return fail(FEMCG_ENOMEM, "bicgstab_solve: host allocation failed");
    } catch (const std::exception &ex) {
        return fail(FEMCG_EDEVICE, "bicgstab_solve: %s", ex.what());
    }
}

}  // extern "C"
