// engine.h -- matrices, workspaces and the slot engine (library internal).
#pragma once

#include <string>

#include "assemble.h"
#include "internal.h"

namespace femcg {

// one device allocation carved into aligned pieces
struct Arena {
    char *base = nullptr;
    size_t size = 0, used = 0;
    void *take(size_t bytes)
    {
        size_t off = (used + 255) & ~(size_t)255;
        used = off + bytes;
        return base ? base + off : nullptr;
    }
};

// per-matrix workspace of one (kp, precision)
struct Work {
    int kp = 0, prec = 0;
    int64_t n = 0;
    int tile_rows = 0, ntiles = 0, ngroups = 0;
    int band = 0;
    int small = 0;  // whole iteration loop in one workgroup (k_solve_small)
    int nt = 0;     // iteration working set beyond the last-level cache: streaming hints
    int lpr = 1;    // SpMM lanes per row at kp = 1 (long rows: 2, 4 or 8)
    // small systems: the matrix padded per workgroup thread,
    // [pass][ell_len][ell_threads/kp]
    int ell_len = 0, ell_threads = 0;
    int32_t *ell_col = nullptr;
    double *ell_v64 = nullptr;
    float *ell_v32 = nullptr;
    double *B64 = nullptr, *X64 = nullptr, *R64 = nullptr, *P64 = nullptr, *Q64 = nullptr;
    float *B32 = nullptr, *X32 = nullptr, *R32 = nullptr, *P32 = nullptr, *Q32 = nullptr;
    double *part64 = nullptr, *part32 = nullptr;
    double *gpart64 = nullptr, *gpart32 = nullptr;
    uint32_t *gtk64 = nullptr, *gtk32 = nullptr;
    char *mem = nullptr;
    size_t bytes = 0;
    ~Work()
    {
        if (mem) (void)hipFree(mem);
    }
};

struct Engine;

// BiCGStab + Block-Jacobi workspace of a matrix (bicgstab.hip): the block
// inverses for one block size, the public -> internal row map, the ten
// solver vectors (internal order), per-block partial dots and the state.
struct BcgWork {
    int bs = 0, grid = 0;
    int64_t n = 0, nb = 0;
    char *mem = nullptr;
    double *binv = nullptr;
    int32_t *iperm = nullptr;
    double *dsc = nullptr;      // row scale, internal order (nullptr: none)
    std::vector<double> scale;  // the caller's row scale, public order (empty: none)
    double *b = nullptr, *x = nullptr, *r = nullptr, *rh = nullptr, *p = nullptr, *ph = nullptr;
    double *v = nullptr, *s = nullptr, *sh = nullptr, *t = nullptr, *part = nullptr;
    void *st = nullptr;         // device state
    void *h_st = nullptr;       // pinned host copy of the state
    double *h_part = nullptr;   // pinned copy of one partial slot
    void *cap = nullptr;        // private capture stream (hipStream_t)
    void *gexec = nullptr;      // graph of one poll window of iterations (hipGraphExec_t)
    size_t bytes = 0;
    double setup_s = 0.0;
    ~BcgWork();
};

}  // namespace femcg

// The opaque handle of the C ABI.
struct fem_matrix {
    femcg::HostSystem hs;
    femcg::SolverCopy sc;
    femcg::DevSparse dev;
    int32_t *d_perm = nullptr;
    // lifting operator K_ID on the device (free rows, Dirichlet columns)
    int32_t *d_lrow = nullptr, *d_lcol = nullptr;
    double *d_lval = nullptr;
    int tile_target = 0;  // 0 = automatic
    int band_mode = -1;   // -1 automatic; 0 tile, 1 band, 2 single-workgroup loop forced
    int band_tile_bytes = 0;  // 0 = automatic
    int lpr_force = 0;        // SpMM lanes per row at kp = 1 (pcg_tune); 0 = from the mean row length
    int max_grid = 2048;
    bool device_assembled = false;
    bool host_only = false;   // FEM_ASSEMBLE_HOST_ONLY: no device copy
    std::map<std::pair<int, int>, std::unique_ptr<femcg::Work>> works;
    std::map<std::pair<int, int>, std::unique_ptr<femcg::Engine>> engines;
    std::unique_ptr<femcg::BcgWork> bcg;
    pcg_stats_t stats{};
    double setup_s = 0.0;
    int last_kp = 0, last_prec = 0;
    ~fem_matrix();
};

namespace femcg {

enum SlotPhase {
    S_FREE = 0,
    S_START,        // needs its first residual
    S_WAIT_START,   // residual launched, waiting for the poll
    S_ITER,         // FP64: iterating in the main table
    S_CHECK,        // FP64: needs the true residual
    S_WAIT_CHECK,
    S_OUTER,        // mixed: needs scale + inner start
    S_WAIT_INNER,   // mixed: inner start launched
    S_INNER,        // mixed: iterating (FP32) in the main table
    S_ACCUM,        // mixed: needs accumulate + outer residual
    S_WAIT_OUTER,
    S_DONE
};

struct Slot {
    SlotPhase ph = S_FREE;
    fem_matrix *A = nullptr;
    Work *w = nullptr;
    int k = 0, kp = 0;
    double tol = 1e-8;
    int64_t max_iter = 0;
    int use_x0 = 0;
    int restarts = 0, outer = 0, max_restarts = 3, max_outer = 30;
    double eta = 1e-4;
    int status = 0;
    bool final_check = false;
    int64_t iters[kMaxK] = {};
    int64_t kernel_iters = 0;      // iterations executed by the kernels (max over columns)
    int64_t kernel_iters32 = 0;
    int64_t outer_residuals = 0;
    double relres[kMaxK] = {};
    int64_t req = -1;              // serving: request id
    int par_off = 0;               // iteration parity offset while in the main table
};

struct Engine {
    int prec = PCG_FP64;
    int max_slots = 1;
    int m = 32;
    int grid = 0;
    bool use_graph = true;
    hipStream_t stream = nullptr;
    // device tables: main (iterating), and the aux tables of one tick
    SysTable *d_main = nullptr, *d_ri64 = nullptr, *d_acc64 = nullptr, *d_acc32 = nullptr,
             *d_sc64 = nullptr, *d_sc32 = nullptr, *d_ri32 = nullptr, *d_small = nullptr;
    SysTable *h_main = nullptr, *h_ri64 = nullptr, *h_acc64 = nullptr, *h_acc32 = nullptr,
             *h_sc64 = nullptr, *h_sc32 = nullptr, *h_ri32 = nullptr, *h_small = nullptr;  // pinned staging
    int small_count[kNumClass] = {};  // systems per kp class in the small table
    int small_res[kNumClass] = {};    // of which with the matrix resident
    SysState *d_st64 = nullptr, *d_st32 = nullptr;
    SysState *h_st64 = nullptr, *h_st32 = nullptr;  // pinned
    std::vector<Slot> slots;
    std::vector<int> main_ids;      // slots in the uploaded main table
    bool main_dirty = true;
    hipGraphExec_t gexec[2] = {nullptr, nullptr};  // chunks starting at an even / odd launch index
    int graph_m = 0, graph_grid = 0;
    unsigned main_mask = 0, graph_mask = 0;  // kp classes present in the main table
    int64_t it_global = 0;          // iterations launched on the main table
    hipStream_t cap = nullptr;
    int64_t replays = 0;
    ~Engine();
};

// ---- functions shared by the ABI files (femcg.cpp, serve.cpp) ----
int fail(int code, const char *fmt, ...);
double now_s();
int pad_k(int k);
int upload_solver_copy(fem_matrix *A);
int upload_lifting(fem_matrix *A);
int get_work(fem_matrix *A, int kp, int prec, Work **out);
size_t work_bytes_estimate(int64_t n, int kp, int prec, int ntiles);
// fem_spmv's tiling and SpMM descriptor without its workspace, for the
// allocation-free product (noalloc.hip), which places the buffers itself:
// spmv_plan fills kp, n, lpr, tile_rows, ntiles, ngroups and band of w (no
// buffer); spmv_desc describes the product on caller-placed buffers; the
// launch uses spmv_grid blocks and the class mask spmv_launch_mask.
void spmv_plan(const fem_matrix *A, int kp, Work &w);
SysDesc spmv_desc(const fem_matrix *A, const Work &w, int k, double *P, double *Q, double *part, double *gpart,
                  uint32_t *gticket, SysState *st);
int spmv_grid(const fem_matrix *A, const Work &w);
unsigned spmv_launch_mask(const Work &w);
size_t matrix_bytes_estimate(const SolverCopy &sc, const HostSystem &hs);
int engine_create(int prec, int max_slots, int m, bool use_graph, std::unique_ptr<Engine> &out);
int engine_admit(Engine *e, int s);
int engine_tick(Engine *e, int *rc_out);
int64_t default_max_iter(int64_t n);
// FEMCG_EINVAL (with the message) for a matrix assembled without a device copy
int require_device(const fem_matrix *A);

}  // namespace femcg
