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
constexpr int kGroup = 64;         // band mode: tiles per reduction group
constexpr int kSmallBlock = 1024;  // small systems: one workgroup runs the whole loop
constexpr int kSmallPass = 4;      // small systems: rows per thread (at kp lanes per row)
constexpr int kSmallElems = kSmallBlock * kSmallPass;  // small systems: n * kp bound (p in LDS)
constexpr int kResBlock = 512;     // small systems with the matrix resident on chip
constexpr int kResPass = kSmallElems / kResBlock;  // rows per thread (at kp lanes per row)
constexpr int kResL = 8;           // entries per row held in registers

// Per-system solver state, resident on the device.
//
// Loop state is double-buffered by iteration parity: iteration i of a system
// reads slot prv = (i & 1) ^ 1 and only the designated block (the one running
// the system's tile 0 of the p-update) writes slot cur = i & 1, so no block
// ever reads a value another block of the same launch writes.  Fields marked
// "host" are copies the host polls; kernels never read them inside the loop.
struct alignas(256) SysState {
    double rho[2][kMaxK];   // r.z of the iterate, by parity
    int32_t active[2][kMaxK];
    int32_t iters[2][kMaxK];
    double bb[kMaxK];       // ||b||^2
    double tol_rel[kMaxK];  // Eq. (2) threshold of each column
    double eta;             // inner systems of iterative refinement: reduction target
    double pad_d;
    double sums[kDots][kMaxK];  // reduced dots of the last producing phase (band mode)
    uint32_t ticket;            // band mode: completed reduction groups of the running phase
    int32_t pad_t;
    int32_t flag[kMaxK];    // 0 normal, 1 disabled (not solved here), FEMCG_EBREAKDOWN
    // host-facing copies
    double rr[kMaxK];       // ||r||^2 of the last residual evaluation
    double relres[kMaxK];   // sqrt(rr / bb) from the last true residual
    int32_t h_iters[kMaxK]; // products A p per column
    int32_t h_active[kMaxK];
    int32_t n_active;       // number of active columns
    int32_t status;         // FEMCG_EBREAKDOWN once any column broke down
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
    int32_t par_off;        // iteration parity of this system = (launch index + par_off) & 1
    int32_t band;           // 0: each block reduces all tile partials at the start of the next
                            //    phase; 1: small tiles swept as a band per XCD, partials
                            //    folded by the blocks that complete each group of tiles
    int64_t tile_base;      // first global tile index of this system
    const int32_t *rowptr;  // CSR [n+1]
    const int64_t *slice_ptr; // SELL [n/C+1]: first entry of each slice
    const int32_t *rowlen;  // SELL [n]: entries of each row
    const int32_t *col;
    const void *val;        // T
    const void *dinv;       // T, inverse diagonal
    const void *b;          // T [n][kp] right-hand side (internal order)
    void *x, *r, *p, *q;    // T [n][kp]
    double *part;           // [kDots][ntiles][kp] per-tile partial dots
    double *gpart;          // band mode: [ngroups][kDots*kp] per-group sums
    uint32_t *gticket;      // band mode: [ngroups] tiles arrived, zero between phases
    SysState *st;
    // single-workgroup systems: entry e of the row served by thread group t
    // in pass i at [(i * ell_len + e) * (ell_threads / kp) + t]; rows padded
    // to ell_len (even) with (own row, 0)
    const int32_t *ell_col;
    const void *ell_val;    // T
    int32_t ell_len;
    int32_t nt;             // 1: x, r, q accessed non-temporally (working set beyond the LLC)
    int32_t ell_threads;    // kSmallBlock (matrix streamed from L2) or kResBlock (resident)
    int32_t lpr;            // SpMM at kp = 1: lanes per row (1, 2, 4 or 8)
};

constexpr int kMaxSys = 256;
constexpr int kNumClass = 7;       // lanes-per-row classes kp = 1, 2, 4, ..., 64
// launch masks: bit c = class c holds systems; kSplitBit = the kp = 1 class
// holds systems whose SpMM splits rows over several lanes (SysDesc.lpr > 1),
// which run in their own SpMM kernel instance (bit 0 then means one-lane
// kp = 1 systems only); kSplitCls names that instance for timed launches
constexpr unsigned kSplitBit = 1u << 7;
constexpr int kSplitCls = 7;

// Systems sorted by kp; class c (kp = 1 << c) owns global tiles
// [cls_begin[c], cls_end[c]).  Each class is processed by its own kernel
// instantiation, specialised on kp.
struct alignas(256) SysTable {
    int32_t nsys;
    int32_t pad;
    int64_t total_tiles;
    int64_t cls_begin[kNumClass];
    int64_t cls_end[kNumClass];
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
// `it` = launch index of the iteration (its parity drives the state slots);
// `cls_mask` = bit c set if class c (kp = 1 << c) has systems in the table.
template <typename T>
void launch_phase(int phase, const SysTable *tab, int grid, int it, int force, unsigned cls_mask,
                  hipStream_t s);
// residual (r = b - A x or r = b), p = D^-1 r, partial b.b r.r r.z; then the
// per-system finalize (one block per system) that decides which columns iterate
template <typename T>
void launch_residual_init(const SysTable *tab, int grid, int nsys, unsigned cls_mask, hipStream_t s);
// One phase of a single-class table (class cls: kp = 1 << cls), with the
// kernel's start and end recorded into ev0 / ev1 by its dispatch packet.
template <typename T>
void launch_phase_timed(int phase, const SysTable *tab, int grid, int it, int force, int cls, hipStream_t s,
                        hipEvent_t ev0, hipEvent_t ev1);
// Small systems (n * kp <= kSmallElems): `niter` iterations, one workgroup
// per system; the table's class ranges index systems, cls_count[c] of them.
// cls_res[c] of the cls_count[c] systems of class c use the resident-matrix
// kernel (ell_threads == kResBlock).
template <typename T>
void launch_small(const SysTable *tab, const int *cls_count, const int *cls_res, int it, int niter, hipStream_t s);
void launch_gather(const double *src, int64_t ld_src, const int32_t *perm, int64_t n, int k,
                   int kp, double *dst, hipStream_t s);
void launch_scatter(const double *src, const int32_t *perm, int64_t n, int k, int kp,
                    const SysState *st, double *dst, hipStream_t s);
void launch_lift(const int32_t *rowptr, const int32_t *col, const double *val, const double *gd,
                 int64_t n, int k, double *B, hipStream_t s);
void launch_ir_scale(const SysTable *tab64, const SysTable *tab32, int grid, hipStream_t s);
void launch_ir_accum(const SysTable *tab64, const SysTable *tab32, int grid, hipStream_t s);

}  // namespace femcg
