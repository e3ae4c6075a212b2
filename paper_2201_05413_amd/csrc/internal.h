// internal.h -- shared declarations of the femcg library (host driver and
// gfx950 kernels).  Not part of the public ABI (that is include/femcg.h).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <map>
#include <memory>
#include <string>
#include <vector>

#include "femcg.h"

namespace femcg {

constexpr int kBlock = 256;        // threads per workgroup: 4 wave64
constexpr int kWave = 64;
constexpr int kMaxK = FEMCG_MAX_K;
constexpr int kDots = 3;           // dot products a kernel may reduce per column
constexpr int kNumXcd = 8;         // MI355X: 8 XCDs x 32 CUs, one L2 each
constexpr int kGroup = 64;         // tiles per first-level reduction group

// Per-system solver scalars, resident on the device.  Every field is written
// only by the single "last tile" of a phase kernel (or by the host between
// solves), so reads in the next kernel see one consistent value.
struct alignas(256) SysState {
    double rho[kMaxK];      // r.z of the current iterate
    double alpha[kMaxK];
    double beta[kMaxK];
    double bb[kMaxK];       // ||b||^2
    double rr[kMaxK];       // ||r||^2 of the last residual evaluation
    double relres[kMaxK];   // sqrt(rr / bb) from the last true residual
    double tol_rel[kMaxK];  // Eq. (2) threshold of each column
    double eta;             // inner systems of iterative refinement: reduction target
    double pad_d;
    int32_t flag[kMaxK];    // 0 normal, 1 disabled (not solved here), FEMCG_EBREAKDOWN
    int32_t active[kMaxK];  // 1 while the column iterates
    int32_t iters[kMaxK];   // products A p since the last reset
    int32_t n_active;       // number of active columns
    int32_t status;         // FEMCG_EBREAKDOWN once any column broke down
    uint32_t ticket;        // arrival counter of the tiles of the running phase
    int32_t pad;
};

// One system as seen by the batched phase kernels.  All pointers are device
// pointers; vectors are [n][kp] in internal (permuted) row order.
struct SysDesc {
    int64_t n;              // rows
    int32_t kp;             // lanes per row = padded column count, power of two
    int32_t k;              // columns in use
    int32_t format;         // FEM_FORMAT_CSR or FEM_FORMAT_SELL
    int32_t sell_shift;     // log2 of the SELL slice height C
    int32_t tile_rows;      // rows per tile (multiple of C and of kBlock/kp)
    int32_t ntiles;
    int32_t use_x;          // residual phase: 1 = r = b - A x, 0 = r = b and x = 0
    int32_t write_p;        // residual phase: 1 = also start p = D^-1 r
    int64_t tile_base;      // first global tile index of this system
    const int32_t *rowptr;  // CSR [n+1]
    const int64_t *slice_ptr; // SELL [n/C+1]: first entry of each slice
    const int32_t *rowlen;  // SELL [n]: entries of each row
    const int32_t *col;
    const void *val;        // T
    const void *dinv;       // T, inverse diagonal
    const void *b;          // T [n][kp] right-hand side (internal order)
    void *x, *r, *p, *q;    // T [n][kp]
    double *part;           // [ntiles][kDots*kp] per-tile partial dots
    double *gpart;          // [ceil(ntiles/kGroup)][kDots*kp] per-group sums
    uint32_t *gticket;      // [ceil(ntiles/kGroup)] arrival counters, zero between phases
    SysState *st;
};

constexpr int kMaxSys = 256;

struct alignas(256) SysTable {
    int32_t nsys;
    int32_t pad;
    int64_t total_tiles;
    SysDesc d[kMaxSys];
};

// ---------------------------------------------------------------------------
// device-side sparse matrix (solver copy) in one precision
// ---------------------------------------------------------------------------
struct DevSparse {
    int format = FEM_FORMAT_CSR;
    int C = 64, sigma = 1;
    int64_t n = 0, nnz = 0, stored = 0;
    int32_t *rowptr = nullptr;
    int64_t *slice_ptr = nullptr;
    int32_t *rowlen = nullptr;
    int32_t *col = nullptr;
    void *val64 = nullptr;   // double
    void *val32 = nullptr;   // float
    void *dinv64 = nullptr;
    void *dinv32 = nullptr;
    size_t bytes = 0;
};

// Kernel launch helpers (kernels.hip).
enum Phase { PH_SPMM = 0, PH_UPDATE = 1, PH_PUPDATE = 2 };

int grid_for(int64_t total_tiles, int max_grid);

// T = double or float.  `tab` is a device SysTable.
template <typename T>
void launch_phase(int phase, const SysTable *tab, int grid, int force, hipStream_t s);
template <typename T>
void launch_residual_init(const SysTable *tab, int grid, hipStream_t s);
void launch_gather(const double *src, int64_t ld_src, const int32_t *perm, int64_t n, int k,
                   int kp, double *dst, hipStream_t s);
void launch_scatter(const double *src, const int32_t *perm, int64_t n, int k, int kp,
                    const SysState *st, double *dst, hipStream_t s);
void launch_lift(const int32_t *rowptr, const int32_t *col, const double *val, const double *gd,
                 int64_t n, int k, double *B, hipStream_t s);
void launch_ir_scale(const SysTable *tab64, const SysTable *tab32, int grid, hipStream_t s);
void launch_ir_accum(const SysTable *tab64, const SysTable *tab32, int grid, hipStream_t s);

}  // namespace femcg
