// noalloc.hip -- the k-column product Y = A X (the SpMM of the iteration)
// without any allocation, for callers that cannot allocate device memory:
// code under HIP graph capture, tight serving loops, harnesses that forbid
// hipMalloc.
//
// Every buffer of fem_spmv beyond the caller's X and Y -- the launch table,
// the loop state, the band-mode group tickets and sums, the per-tile partial
// dots, and the permuted / padded copies P of X and Q of Y -- is carved out
// of one fixed device array, `scratch`, of kNoallocScratchBytes.  The host
// never names that array in device work: the first call on a device takes
// its address there with hipGetSymbolAddress (each device holds its own copy
// at its own address) and every kernel argument and descriptor is derived
// from that address.  The table and state are written by a small kernel that
// receives the descriptor by value, so the call issues no host copy either
// and is fully asynchronous on the caller's stream.
//
// The kernels are fem_spmv's (gather to the solver copy's row order, the
// SpMM phase kernel, scatter back) with the same tiling, so Y is identical
// to fem_spmv's bit for bit.
#include "engine.h"

#include <mutex>

namespace femcg {

constexpr size_t kNoallocScratchBytes = FEMCG_NOALLOC_SCRATCH_BYTES;  // per device, held until the process ends
constexpr int kNoallocMaxDevices = 64;

}  // namespace femcg

static __device__ __align__(256) char scratch[femcg::kNoallocScratchBytes];

namespace femcg {
namespace {

std::mutex g_scratch_mu;
void *g_scratch_ptr[kNoallocMaxDevices] = {};

// Device address of `scratch` on the current device (taken once per device).
int scratch_address(void **out)
{
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return fail(FEMCG_EDEVICE, "hipGetDevice: %s", hipGetErrorString(e));
    if (dev < 0 || dev >= kNoallocMaxDevices) return fail(FEMCG_EDEVICE, "device ordinal %d out of range", dev);
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(FEMCG_EDEVICE, "hipGetSymbolAddress(scratch) on device %d: %s", dev, hipGetErrorString(e));
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return FEMCG_OK;
}

// Byte offsets of the pieces inside the scratch array, 256-byte aligned.
struct Layout {
    size_t tab = 0, st = 0, gtk = 0, gpart = 0, part = 0, P = 0, Q = 0, end = 0;
};

size_t take(size_t &used, size_t bytes)
{
    const size_t off = (used + 255) & ~(size_t)255;
    used = off + bytes;
    return off;
}

Layout layout_of(const Work &w)
{
    Layout L;
    size_t used = 0;
    const size_t nv = (size_t)std::max<int64_t>(w.n, 1) * w.kp;
    L.tab = take(used, offsetof(SysTable, d) + sizeof(SysDesc));
    L.st = take(used, sizeof(SysState));
    L.gtk = take(used, (size_t)w.ngroups * sizeof(uint32_t));
    L.gpart = take(used, (size_t)w.ngroups * kDots * w.kp * sizeof(double));
    L.part = take(used, (size_t)w.ntiles * kDots * w.kp * sizeof(double));
    L.P = take(used, nv * sizeof(double));
    L.Q = take(used, nv * sizeof(double));
    L.end = used;
    return L;
}

// One workgroup: the single-system launch table, and zeros in the loop state
// and the band-mode group tickets (the previous call's contents are still in
// the array; the SpMM runs with force = 1, so the state's contents other than
// its ticket do not matter, but all of it is cleared).
__global__ __launch_bounds__(kBlock) void k_noalloc_setup(SysTable *tab, SysDesc D, int cls, SysState *st,
                                                          uint32_t *gtk, int ngroups)
{
    if (threadIdx.x == 0) {
        tab->nsys = 1;
        tab->pad = 0;
        tab->total_tiles = D.ntiles;
        for (int c = 0; c < kNumClass; ++c) {
            tab->cls_begin[c] = 0;
            tab->cls_end[c] = c == cls ? D.ntiles : 0;
        }
        tab->d[0] = D;
    }
    uint32_t *w = reinterpret_cast<uint32_t *>(st);
    for (size_t i = threadIdx.x; i < sizeof(SysState) / sizeof(uint32_t); i += blockDim.x) w[i] = 0u;
    for (int g = threadIdx.x; g < ngroups; g += blockDim.x) gtk[g] = 0u;
}

int class_index(int kp)
{
    int c = 0;
    while ((1 << c) < kp) ++c;
    return c;
}

}  // namespace
}  // namespace femcg

using namespace femcg;

extern "C" int fem_spmv_noalloc(fem_matrix *A, const double *X, double *Y, int32_t k, void *stream)
{
    if (!A || !X || !Y) return fail(FEMCG_EINVAL, "NULL argument");
    if (int rc = require_device(A)) return rc;
    if (k < 1 || k > kMaxK) return fail(FEMCG_EUNSUPPORTED, "k=%d outside 1..%d", k, kMaxK);
    const int kp = pad_k(k);
    Work w;
    spmv_plan(A, kp, w);
    const Layout L = layout_of(w);
    if (L.end > kNoallocScratchBytes)
        return fail(FEMCG_EINVAL,
                    "fem_spmv_noalloc: n = %lld rows x %d lanes needs %zu bytes of scratch, above the fixed %zu "
                    "(about n * kp <= %zu); use fem_spmv",
                    (long long)w.n, kp, L.end, kNoallocScratchBytes, kNoallocScratchBytes / 16);
    void *base = nullptr;
    if (int rc = scratch_address(&base)) return rc;
    char *b = static_cast<char *>(base);
    auto *tab = reinterpret_cast<SysTable *>(b + L.tab);
    auto *st = reinterpret_cast<SysState *>(b + L.st);
    auto *gtk = reinterpret_cast<uint32_t *>(b + L.gtk);
    auto *gpart = reinterpret_cast<double *>(b + L.gpart);
    auto *part = reinterpret_cast<double *>(b + L.part);
    auto *P = reinterpret_cast<double *>(b + L.P);
    auto *Q = reinterpret_cast<double *>(b + L.Q);
    hipStream_t s = (hipStream_t)stream;
    const SysDesc D = spmv_desc(A, w, k, P, Q, part, gpart, gtk, st);
    hipLaunchKernelGGL(k_noalloc_setup, dim3(1), dim3(kBlock), 0, s, tab, D, class_index(kp), st, gtk, w.ngroups);
    launch_gather(X, k, A->d_perm, w.n, k, kp, P, s);
    launch_phase<double>(PH_SPMM, tab, spmv_grid(A, w), 0, 1, spmv_launch_mask(w), s);
    launch_scatter(Q, A->d_perm, w.n, k, kp, nullptr, Y, s);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(FEMCG_EDEVICE, "fem_spmv_noalloc launch: %s", hipGetErrorString(e));
    return FEMCG_OK;
}
