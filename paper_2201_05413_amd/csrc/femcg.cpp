// femcg.cpp -- host driver and C ABI of the MI355X Jacobi-PCG library.
//
// A solve is a sequence of "ticks" of a slot engine.  Each resident system
// (a slot) walks a small state machine -- start residual, iterate, confirm the
// Eq. (2) test with the true FP64 residual, restart or finish; for the mixed
// precision form also scale/accumulate the FP32 inner corrections -- and each
// tick launches, for all slots at once: the transition kernels of the slots
// that changed state, then `check_every` PCG iterations of every iterating
// slot (a HIP graph of 3 persistent launches per iteration over the device
// system table), then one device-to-host copy of the per-slot states.
// pcg_solve is an engine with one slot; pcg_solve_batch and the server use
// the same engine with many.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <cstdlib>
#include <deque>
#include <exception>
#include <new>
#include <functional>
#include <mutex>

#include "engine.h"

namespace femcg {

// ---------------------------------------------------------------------------
// errors
// ---------------------------------------------------------------------------
static thread_local std::string g_err;

int fail(int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

#define HIPCHK(call)                                                                        \
    do {                                                                                    \
        hipError_t e_ = (call);                                                             \
        if (e_ != hipSuccess) return fail(FEMCG_EDEVICE, "%s: %s", #call, hipGetErrorString(e_)); \
    } while (0)

double now_s()
{
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

static int ilog2(int v)
{
    int s = 0;
    while ((1 << s) < v) ++s;
    return s;
}

int pad_k(int k)
{
    int kp = 1;
    while (kp < k) kp <<= 1;
    return kp;
}

static void free_dev(fem_matrix *A)
{
    DevSparse &d = A->dev;
    void *ptrs[] = {d.rowptr, d.slice_ptr, d.rowlen, d.col, d.val64, d.val32, d.dinv64, d.dinv32};
    for (void *p : ptrs)
        if (p) (void)hipFree(p);
    d = DevSparse{};
}

template <typename T, typename Al>
static int upload(T **dst, const std::vector<T, Al> &src)
{
    *dst = nullptr;
    if (src.empty()) return FEMCG_OK;
    HIPCHK(hipMalloc((void **)dst, sizeof(T) * src.size()));
    HIPCHK(hipMemcpy(*dst, src.data(), sizeof(T) * src.size(), hipMemcpyHostToDevice));
    return FEMCG_OK;
}

int upload_solver_copy(fem_matrix *A)
{
    free_dev(A);
    A->works.clear();
    A->engines.clear();
    A->bcg.reset();
    const SolverCopy &sc = A->sc;
    DevSparse &d = A->dev;
    d.format = sc.format;
    d.C = sc.C;
    d.sigma = sc.sigma;
    d.n = sc.n;
    d.nnz = sc.nnz;
    d.stored = sc.stored;
    int rc;
    const BigVec<double> &v64 = sc.format == FEM_FORMAT_SELL ? sc.sell_val : sc.val;
    std::vector<float> v32(v64.size()), di32(sc.dinv.size());
    parallel_for((int64_t)v64.size(), [&](int64_t a, int64_t b) {
        for (int64_t i = a; i < b; ++i) v32[i] = (float)v64[i];
    });
    for (size_t i = 0; i < sc.dinv.size(); ++i) di32[i] = (float)sc.dinv[i];
    if (sc.format == FEM_FORMAT_SELL) {
        if ((rc = upload(&d.slice_ptr, sc.slice_ptr))) return rc;
        if ((rc = upload(&d.rowlen, sc.rowlen))) return rc;
        if ((rc = upload(&d.col, sc.sell_col))) return rc;
    } else {
        if ((rc = upload(&d.rowptr, sc.rowptr))) return rc;
        if ((rc = upload(&d.col, sc.col))) return rc;
    }
    double *v64d = nullptr, *di64d = nullptr;
    float *v32d = nullptr, *di32d = nullptr;
    if ((rc = upload(&v64d, v64))) return rc;
    if ((rc = upload(&v32d, v32))) return rc;
    if ((rc = upload(&di64d, sc.dinv))) return rc;
    if ((rc = upload(&di32d, di32))) return rc;
    d.val64 = v64d;
    d.val32 = v32d;
    d.dinv64 = di64d;
    d.dinv32 = di32d;
    d.bytes = sc.stored * (4 + 8 + 4) + sc.n * (8 + 4) +
              (sc.format == FEM_FORMAT_SELL ? sc.slice_ptr.size() * 8 + sc.n * 4 : (sc.n + 1) * 4);
    if (A->d_perm) (void)hipFree(A->d_perm);
    if ((rc = upload(&A->d_perm, sc.perm))) return rc;
    return FEMCG_OK;
}

// Tiling of one system.  Small systems: large tiles whose partials every
// block of the next phase reduces at its start.  Large systems (band mode):
// small tiles that the blocks of each XCD sweep as one band, so rows that
// share gathered neighbours are processed close in time on the same L2.
// SpMM lanes per row at kp = 1, from the mean kept row length: long rows
// (P2-P4) are split over 2, 4 or 8 lanes, so each lane's chain of dependent
// index, value and gather loads shortens (measured on a 2D mesh of 86k
// vertices: P2 -4%, P3 -19%, P4 -32% time-to-tol; P1 rows, 7 entries on
// average, stay on one lane).
static int choose_lpr(const fem_matrix *A, int kp)
{
    if (kp != 1) return 1;
    const double mean = A->sc.n ? (double)A->sc.nnz / (double)A->sc.n : 0.0;
    int lpr = mean >= 32.0 ? 8 : (mean >= 14.0 ? 4 : (mean >= 8.0 ? 2 : 1));
    if (A->lpr_force > 0) lpr = A->lpr_force;                       // pcg_tune's choice
    if (const char *ev = std::getenv("FEMCG_LPR")) lpr = atoi(ev);  // tuning override
    return (lpr == 2 || lpr == 4 || lpr == 8) ? lpr : 1;
}

static void choose_tiles(const fem_matrix *A, int kp, int lpr, int &tile_rows, int &ntiles, int &band)
{
    const int64_t n = A->dev.n;
    const int rps = kBlock / kp;
    const int unit = std::max(rps, A->dev.format == FEM_FORMAT_SELL ? A->dev.C : 1);
    const double vec_bytes = (double)n * kp * 8.0;
    // vectors beyond the last-level cache: thin band tiles keep each XCD's
    // working window of P compact and let the dispatcher balance tiles
    band = (A->band_mode == 0 || A->band_mode == 1) ? A->band_mode : (vec_bytes > 64e6 ? 1 : 0);
    if (const char *ev = std::getenv("FEMCG_BAND")) band = atoi(ev);  // tuning override
    int64_t rows;
    if (band) {
        // automatic: about 4096 tiles (enough blocks to fill the chip with one
        // tile each), 16..64 KB of one vector per tile
        int tb = A->band_tile_bytes;
        if (tb <= 0) {
            tb = 16384;
            while (tb < 65536 && vec_bytes / (2.0 * tb) >= 4096.0) tb *= 2;
        }
        if (const char *ev = std::getenv("FEMCG_BAND_TILE_BYTES")) tb = std::max(1024, atoi(ev));
        rows = std::max<int64_t>(1, tb / (kp * 8));
    } else {
        // every block reduces all tile partials at the start of a phase, so
        // keep ntiles * kp bounded (<= 16K partials per dot); split rows
        // (lpr > 1 lanes per row) take 4096 tiles, so that a block's serial
        // batches stay few
        int target = A->tile_target > 0 ? A->tile_target
                                        : (lpr > 1 ? 4096 : std::max(256, std::min(1024, 16384 / kp)));
        if (const char *ev = std::getenv("FEMCG_TILE_TARGET")) target = std::max(1, atoi(ev));  // tuning override
        rows = (n + target - 1) / target;
    }
    rows = ((rows + unit - 1) / unit) * unit;
    if (rows < unit) rows = unit;
    if (rows > (1 << 30)) rows = 1 << 30;
    tile_rows = (int)rows;
    ntiles = (int)((n + rows - 1) / rows);
}

// Grid cap for a launch over systems of this matrix.  Band tiles carry no
// per-block reduction prologue, so they run one tile per block at up to four
// times the resident grid: the hardware dispatcher then balances the uneven
// gather cost of the tiles, which a static tile split cannot.
static int grid_cap(const fem_matrix *A, const Work *w)
{
    return (w && w->band) ? 4 * A->max_grid : A->max_grid;
}

int get_work(fem_matrix *A, int kp, int prec, Work **out)
{
    if (int rc = require_device(A)) return rc;
    auto key = std::make_pair(kp, prec);
    auto it = A->works.find(key);
    if (it != A->works.end()) {
        *out = it->second.get();
        return FEMCG_OK;
    }
    auto w = std::make_unique<Work>();
    w->kp = kp;
    w->prec = prec;
    w->n = A->dev.n;
    w->lpr = choose_lpr(A, kp);
    choose_tiles(A, kp, w->lpr, w->tile_rows, w->ntiles, w->band);
    const bool fits_small = w->n * kp <= kSmallElems;
    if (A->band_mode == 2 && !fits_small)
        return fail(FEMCG_EINVAL, "single-workgroup mode needs n * kp <= %d (n = %lld, kp = %d)", kSmallElems,
                    (long long)w->n, kp);
    w->small = A->band_mode == 2 || (A->band_mode == -1 && fits_small);
    {
        // one iteration touches the matrix, x, r, p, q and D^-1; the MI355X
        // last-level (Infinity) cache holds 256 MB
        const double sv = prec == PCG_FP64 ? 8.0 : 4.0;
        const double vb = (double)w->n * kp * sv;
        const double mb = (double)A->sc.stored * (sv + 4.0);
        w->nt = (mb + 4.0 * vb + (double)w->n * sv) > 256e6 ? 1 : 0;
        if (const char *ev = std::getenv("FEMCG_NT")) w->nt = atoi(ev);  // tuning override
    }
    if (const char *ev = std::getenv("FEMCG_SMALL")) w->small = w->small && atoi(ev) != 0;  // tuning override

    w->ngroups = (w->ntiles + kGroup - 1) / kGroup;
    const size_t nv = (size_t)std::max<int64_t>(w->n, 1) * kp;
    const size_t np = (size_t)w->ntiles * kDots * kp, ngp = (size_t)w->ngroups * kDots * kp;
    // small systems: ELL layout of the solver copy per workgroup thread group;
    // rows of at most kResL entries keep the matrix resident (512 threads)
    if (w->small) {
        int64_t L = 1;
        for (int64_t i = 0; i < w->n; ++i) L = std::max<int64_t>(L, A->sc.rowptr[i + 1] - A->sc.rowptr[i]);
        w->ell_len = (int)((L + 1) / 2 * 2);
        w->ell_threads = w->ell_len <= kResL ? kResBlock : kSmallBlock;
        if (const char *ev = std::getenv("FEMCG_SMALL_RES")) {  // tuning override
            if (atoi(ev) == 0) w->ell_threads = kSmallBlock;
        }
    }
    const int rpp = w->small ? w->ell_threads / kp : 1;
    const int npass = w->small ? (int)((w->n + rpp - 1) / rpp) : 0;
    const size_t ne = (size_t)npass * w->ell_len * rpp;
    Arena ar;
    for (int pass = 0; pass < 2; ++pass) {
        ar.used = 0;
        w->B64 = (double *)ar.take(nv * 8);
        w->X64 = (double *)ar.take(nv * 8);
        w->R64 = (double *)ar.take(nv * 8);
        if (prec == PCG_FP64) {
            w->P64 = (double *)ar.take(nv * 8);
            w->Q64 = (double *)ar.take(nv * 8);
        } else {
            w->B32 = (float *)ar.take(nv * 4);
            w->X32 = (float *)ar.take(nv * 4);
            w->R32 = (float *)ar.take(nv * 4);
            w->P32 = (float *)ar.take(nv * 4);
            w->Q32 = (float *)ar.take(nv * 4);
            w->part32 = (double *)ar.take(np * 8);
            w->gpart32 = (double *)ar.take(ngp * 8);
            w->gtk32 = (uint32_t *)ar.take((size_t)w->ngroups * 4);
        }
        w->part64 = (double *)ar.take(np * 8);
        w->gpart64 = (double *)ar.take(ngp * 8);
        w->gtk64 = (uint32_t *)ar.take((size_t)w->ngroups * 4);
        if (ne) {
            w->ell_col = (int32_t *)ar.take(ne * 4);
            w->ell_v64 = (double *)ar.take(ne * 8);
            w->ell_v32 = (float *)ar.take(ne * 4);
        }
        if (pass == 0) {
            ar.size = ar.used;
            if (hipMalloc((void **)&ar.base, ar.size) != hipSuccess)
                return fail(FEMCG_ENOMEM, "device workspace of %zu bytes", ar.size);
            HIPCHK(hipMemset(ar.base, 0, ar.size));
        }
    }
    w->mem = ar.base;
    w->bytes = ar.size;
    if (ne) {
        std::vector<int32_t> ec(ne);
        std::vector<double> ev(ne);
        std::vector<float> ef(ne);
        for (int i = 0; i < npass; ++i)
            for (int t = 0; t < rpp; ++t) {
                const int64_t row = (int64_t)i * rpp + t;
                const int64_t b = row < w->n ? A->sc.rowptr[row] : 0;
                const int64_t len = row < w->n ? A->sc.rowptr[row + 1] - b : 0;
                for (int e = 0; e < w->ell_len; ++e) {
                    const size_t o = ((size_t)i * w->ell_len + e) * rpp + t;
                    ec[o] = e < len ? A->sc.col[b + e] : (row < w->n ? (int32_t)row : 0);
                    ev[o] = e < len ? A->sc.val[b + e] : 0.0;
                    ef[o] = (float)ev[o];
                }
            }
        HIPCHK(hipMemcpy(w->ell_col, ec.data(), ne * 4, hipMemcpyHostToDevice));
        HIPCHK(hipMemcpy(w->ell_v64, ev.data(), ne * 8, hipMemcpyHostToDevice));
        HIPCHK(hipMemcpy(w->ell_v32, ef.data(), ne * 4, hipMemcpyHostToDevice));
    }
    *out = w.get();
    A->works[key] = std::move(w);
    return FEMCG_OK;
}

size_t work_bytes_estimate(int64_t n, int kp, int prec, int ntiles)
{
    const size_t nv = (size_t)std::max<int64_t>(n, 1) * kp;
    const size_t parts = (size_t)ntiles * kDots * kp * 8 * 2;
    const size_t vec = prec == PCG_FP64 ? nv * 8 * 5 : nv * (8 * 3 + 4 * 5);
    return vec + parts * (prec == PCG_FP64 ? 1 : 2) + 16 * 256;
}

size_t matrix_bytes_estimate(const SolverCopy &sc, const HostSystem &hs)
{
    const size_t idx = sc.format == FEM_FORMAT_SELL ? sc.slice_ptr.size() * 8 + sc.n * 4 : (sc.n + 1) * 4;
    return (size_t)sc.stored * (4 + 8 + 4) + (size_t)sc.n * (8 + 4 + 4) + idx +
           hs.l_col.size() * 12 + hs.l_rowptr.size() * 4;
}

static SysDesc make_desc_base(const fem_matrix *A, const Work *w, bool fp32, const void *b, void *x, void *r,
                              void *p, void *q, double *part, SysState *st, int k);

static SysDesc make_desc(const fem_matrix *A, const Work *w, bool fp32, const void *b, void *x, void *r,
                         void *p, void *q, double *part, SysState *st, int k)
{
    SysDesc D = make_desc_base(A, w, fp32, b, x, r, p, q, part, st, k);
    D.band = w->band;
    D.ell_col = w->ell_col;
    D.ell_val = fp32 ? (const void *)w->ell_v32 : (const void *)w->ell_v64;
    D.ell_len = w->ell_len;
    D.ell_threads = w->ell_threads;
    D.nt = w->nt;
    D.lpr = w->lpr;
    D.gpart = fp32 ? w->gpart32 : w->gpart64;
    D.gticket = fp32 ? w->gtk32 : w->gtk64;
    return D;
}

static SysDesc make_desc_base(const fem_matrix *A, const Work *w, bool fp32, const void *b, void *x, void *r,
                              void *p, void *q, double *part, SysState *st, int k)
{
    SysDesc D{};
    const DevSparse &d = A->dev;
    D.n = d.n;
    D.kp = w->kp;
    D.k = k;
    D.format = d.format;
    D.sell_shift = ilog2(d.C);
    D.tile_rows = w->tile_rows;
    D.ntiles = w->ntiles;
    D.rowptr = d.rowptr;
    D.slice_ptr = d.slice_ptr;
    D.rowlen = d.rowlen;
    D.col = d.col;
    D.val = fp32 ? d.val32 : d.val64;
    D.dinv = fp32 ? d.dinv32 : d.dinv64;
    D.b = b;
    D.x = x;
    D.r = r;
    D.p = p;
    D.q = q;
    D.part = part;
    D.st = st;
    return D;
}

Engine::~Engine()
{
    for (auto &g : gexec)
        if (g) (void)hipGraphExecDestroy(g);
    if (cap) (void)hipStreamDestroy(cap);
    SysTable *dt[] = {d_main, d_ri64, d_acc64, d_acc32, d_sc64, d_sc32, d_ri32, d_small};
    for (auto p : dt)
        if (p) (void)hipFree(p);
    SysTable *ht[] = {h_main, h_ri64, h_acc64, h_acc32, h_sc64, h_sc32, h_ri32, h_small};
    for (auto p : ht)
        if (p) (void)hipHostFree(p);
    if (d_st64) (void)hipFree(d_st64);
    if (d_st32) (void)hipFree(d_st32);
    if (h_st64) (void)hipHostFree(h_st64);
    if (h_st32) (void)hipHostFree(h_st32);
}


static size_t table_bytes(int nsys)
{
    return offsetof(SysTable, d) + sizeof(SysDesc) * (size_t)std::max(nsys, 1);
}

int engine_create(int prec, int max_slots, int m, bool use_graph, std::unique_ptr<Engine> &out)
{
    auto e = std::make_unique<Engine>();
    e->prec = prec;
    e->max_slots = std::min(max_slots, kMaxSys);
    e->m = std::max(1, m);
    e->use_graph = use_graph;
    e->slots.resize(e->max_slots);
    const size_t tb = table_bytes(e->max_slots);
    SysTable **dts[] = {&e->d_main, &e->d_ri64, &e->d_acc64, &e->d_acc32, &e->d_sc64, &e->d_sc32, &e->d_ri32,
                        &e->d_small};
    SysTable **hts[] = {&e->h_main, &e->h_ri64, &e->h_acc64, &e->h_acc32, &e->h_sc64, &e->h_sc32, &e->h_ri32,
                        &e->h_small};
    for (auto p : dts) {
        HIPCHK(hipMalloc((void **)p, tb));
        HIPCHK(hipMemset(*p, 0, tb));
    }
    for (auto p : hts) {
        HIPCHK(hipHostMalloc((void **)p, tb, hipHostMallocDefault));
        std::memset(*p, 0, tb);
    }
    HIPCHK(hipMalloc((void **)&e->d_st64, sizeof(SysState) * e->max_slots));
    HIPCHK(hipMalloc((void **)&e->d_st32, sizeof(SysState) * e->max_slots));
    HIPCHK(hipMemset(e->d_st64, 0, sizeof(SysState) * e->max_slots));
    HIPCHK(hipMemset(e->d_st32, 0, sizeof(SysState) * e->max_slots));
    HIPCHK(hipHostMalloc((void **)&e->h_st64, sizeof(SysState) * e->max_slots, hipHostMallocDefault));
    HIPCHK(hipHostMalloc((void **)&e->h_st32, sizeof(SysState) * e->max_slots, hipHostMallocDefault));
    std::memset(e->h_st64, 0, sizeof(SysState) * e->max_slots);
    std::memset(e->h_st32, 0, sizeof(SysState) * e->max_slots);
    HIPCHK(hipStreamCreateWithFlags(&e->cap, hipStreamNonBlocking));
    out = std::move(e);
    return FEMCG_OK;
}

static SysDesc slot_desc(Engine *e, int s, bool fp32)
{
    Slot &sl = e->slots[s];
    Work *w = sl.w;
    if (!fp32)
        return make_desc(sl.A, w, false, w->B64, w->X64, w->R64, w->P64, w->Q64, w->part64, e->d_st64 + s,
                         sl.k);
    return make_desc(sl.A, w, true, w->B32, w->X32, w->R32, w->P32, w->Q32, w->part32, e->d_st32 + s, sl.k);
}

static int class_of(int kp)
{
    int c = 0;
    while ((1 << c) < kp) ++c;
    return c;
}

// launch-mask bit of one system: its kp class, or the split-row kp = 1 bit
static unsigned launch_bit(int kp, int lpr)
{
    return (kp == 1 && lpr > 1) ? kSplitBit : 1u << class_of(kp);
}

// Fill a host table from slot ids (sorted by kp class in place, stable, with
// their per-system flags); returns total tiles and the class mask.
static int64_t fill_table(Engine *e, SysTable *h, std::vector<int> &ids, bool fp32, int use_x, int write_p,
                          unsigned *mask, std::vector<int> *use_x_per = nullptr)
{
    std::vector<int> ux(ids.size(), use_x);
    if (use_x_per) ux = *use_x_per;
    std::vector<size_t> ord(ids.size());
    for (size_t i = 0; i < ord.size(); ++i) ord[i] = i;
    std::stable_sort(ord.begin(), ord.end(),
                     [&](size_t a, size_t b) { return e->slots[ids[a]].kp < e->slots[ids[b]].kp; });
    std::vector<int> sid(ids.size()), sux(ids.size());
    for (size_t i = 0; i < ord.size(); ++i) {
        sid[i] = ids[ord[i]];
        sux[i] = ux[ord[i]];
    }
    ids = sid;
    if (use_x_per) *use_x_per = sux;
    int64_t base = 0;
    unsigned m = 0, seen = 0;
    for (int c = 0; c < kNumClass; ++c) h->cls_begin[c] = h->cls_end[c] = 0;
    h->nsys = (int)ids.size();
    for (size_t i = 0; i < ids.size(); ++i) {
        SysDesc D = slot_desc(e, ids[i], fp32);
        D.tile_base = base;
        D.use_x = sux[i];
        D.write_p = write_p;
        D.par_off = e->slots[ids[i]].par_off;
        const int c = class_of(D.kp);
        if (!(seen & (1u << c))) h->cls_begin[c] = base;
        seen |= 1u << c;
        m |= launch_bit(D.kp, D.lpr);
        base += D.ntiles;
        h->cls_end[c] = base;
        h->d[i] = D;
    }
    h->total_tiles = base;
    if (mask) *mask = m;
    return base;
}

// Table of single-workgroup systems: class c owns system indices
// [cls_begin[c], cls_end[c]) (ids sorted by kp), one workgroup each.
static void fill_small_table(Engine *e, SysTable *h, const std::vector<int> &ids, bool fp32)
{
    for (int c = 0; c < kNumClass; ++c) {
        h->cls_begin[c] = h->cls_end[c] = 0;
        e->small_count[c] = 0;
        e->small_res[c] = 0;
    }
    h->nsys = (int)ids.size();
    h->total_tiles = 0;
    for (size_t i = 0; i < ids.size(); ++i) {
        SysDesc D = slot_desc(e, ids[i], fp32);
        D.tile_base = 0;
        D.par_off = e->slots[ids[i]].par_off;
        const int c = class_of(D.kp);
        if (e->small_count[c] == 0) h->cls_begin[c] = (int64_t)i;
        e->small_count[c]++;
        e->small_res[c] += D.ell_threads == kResBlock;
        h->cls_end[c] = (int64_t)i + 1;
        h->d[i] = D;
    }
}

static void set_single_table(SysTable *h, const SysDesc &D)
{
    h->nsys = 1;
    h->total_tiles = D.ntiles;
    for (int c = 0; c < kNumClass; ++c) h->cls_begin[c] = h->cls_end[c] = 0;
    const int c = class_of(D.kp);
    h->cls_end[c] = D.ntiles;
    h->d[0] = D;
}

static int upload_table(Engine *e, SysTable *d, SysTable *h)
{
    HIPCHK(hipMemcpyAsync(d, h, table_bytes(h->nsys), hipMemcpyHostToDevice, e->stream));
    return FEMCG_OK;
}

// `iters` iterations on the main table; launch indices it0, it0+1, ...
static int launch_iterations(Engine *e, int iters, int grid, int64_t it0)
{
    const unsigned m = e->main_mask;
    for (int i = 0; i < iters; ++i) {
        const int it = (int)((it0 + i) & 1);
        if (e->prec == PCG_FP64) {
            launch_phase<double>(PH_SPMM, e->d_main, grid, it, 0, m, e->stream);
            launch_phase<double>(PH_UPDATE, e->d_main, grid, it, 0, m, e->stream);
            launch_phase<double>(PH_PUPDATE, e->d_main, grid, it, 0, m, e->stream);
        } else {
            launch_phase<float>(PH_SPMM, e->d_main, grid, it, 0, m, e->stream);
            launch_phase<float>(PH_UPDATE, e->d_main, grid, it, 0, m, e->stream);
            launch_phase<float>(PH_PUPDATE, e->d_main, grid, it, 0, m, e->stream);
        }
    }
    HIPCHK(hipGetLastError());
    return FEMCG_OK;
}

// Graphs of m iterations for chunks starting at an even / odd launch index.
static int ensure_graph(Engine *e, int grid)
{
    if (e->gexec[0] && e->graph_m == e->m && e->graph_grid == grid && e->graph_mask == e->main_mask)
        return FEMCG_OK;
    for (auto &g : e->gexec)
        if (g) {
            HIPCHK(hipGraphExecDestroy(g));
            g = nullptr;
        }
    for (int par = 0; par < 2; ++par) {
        hipGraph_t g = nullptr;
        HIPCHK(hipStreamBeginCapture(e->cap, hipStreamCaptureModeThreadLocal));
        hipStream_t saved = e->stream;
        e->stream = e->cap;
        int rc = launch_iterations(e, e->m, grid, par);
        e->stream = saved;
        hipError_t ce = hipStreamEndCapture(e->cap, &g);
        if (rc) return rc;
        if (ce != hipSuccess) return fail(FEMCG_EDEVICE, "graph capture: %s", hipGetErrorString(ce));
        hipError_t ie = hipGraphInstantiate(&e->gexec[par], g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (ie != hipSuccess) return fail(FEMCG_EDEVICE, "graph instantiate: %s", hipGetErrorString(ie));
    }
    e->graph_m = e->m;
    e->graph_grid = grid;
    e->graph_mask = e->main_mask;
    return FEMCG_OK;
}

static void init_state(SysState &st, int k, int kp, double tol, double eta)
{
    std::memset(&st, 0, sizeof st);
    for (int j = 0; j < kMaxK; ++j) {
        st.tol_rel[j] = tol;
        st.flag[j] = j < k ? 0 : 1;
    }
    st.eta = eta;
    (void)kp;
}

// Admit a slot: state reset.  B/X already gathered into the work buffers.
int engine_admit(Engine *e, int s)
{
    Slot &sl = e->slots[s];
    SysState st;
    init_state(st, sl.k, sl.kp, sl.tol, sl.eta);
    HIPCHK(hipMemcpyAsync(e->d_st64 + s, &st, sizeof st, hipMemcpyHostToDevice, e->stream));
    if (e->prec == PCG_MIXED) {
        SysState st2;
        init_state(st2, sl.k, sl.kp, 1.0, sl.eta);
        HIPCHK(hipMemcpyAsync(e->d_st32 + s, &st2, sizeof st2, hipMemcpyHostToDevice, e->stream));
    }
    // the memcpy source is a stack object: make the copy complete before returning
    HIPCHK(hipStreamSynchronize(e->stream));
    sl.ph = S_START;
    sl.status = 0;
    sl.restarts = 0;
    sl.outer = 0;
    sl.final_check = false;
    sl.kernel_iters = sl.kernel_iters32 = sl.outer_residuals = 0;
    std::fill(sl.iters, sl.iters + kMaxK, 0);
    e->main_dirty = true;
    return FEMCG_OK;
}

static int64_t slot_max_iters(const Slot &sl)
{
    int64_t m = 0;
    for (int j = 0; j < sl.k; ++j) m = std::max(m, sl.iters[j]);
    return m;
}

// One tick of the engine.  Returns the number of slots not yet done.
int engine_tick(Engine *e, int *rc_out)
{
    *rc_out = 0;
    const bool mixed = e->prec == PCG_MIXED;
    std::vector<int> ri64, ri64_usex, acc, sc;
    for (int s = 0; s < e->max_slots; ++s) {
        Slot &sl = e->slots[s];
        switch (sl.ph) {
        case S_START:
            ri64.push_back(s);
            ri64_usex.push_back(sl.use_x0);
            sl.ph = S_WAIT_START;
            break;
        case S_CHECK:
            ri64.push_back(s);
            ri64_usex.push_back(1);
            sl.ph = S_WAIT_CHECK;
            break;
        case S_OUTER:
            sc.push_back(s);
            sl.ph = S_WAIT_INNER;
            break;
        case S_ACCUM:
            acc.push_back(s);
            ri64.push_back(s);
            ri64_usex.push_back(1);
            sl.ph = S_WAIT_OUTER;
            break;
        default:
            break;
        }
    }
    int rc;
    // 1. transition kernels
    if (!acc.empty()) {
        int64_t T = fill_table(e, e->h_acc64, acc, false, 1, 0, nullptr);
        fill_table(e, e->h_acc32, acc, true, 0, 0, nullptr);
        if ((rc = upload_table(e, e->d_acc64, e->h_acc64)) || (rc = upload_table(e, e->d_acc32, e->h_acc32))) {
            *rc_out = rc;
            return -1;
        }
        launch_ir_accum(e->d_acc64, e->d_acc32, grid_for(T, 2048), e->stream);
    }
    if (!ri64.empty()) {
        unsigned m;
        int64_t T = fill_table(e, e->h_ri64, ri64, false, 0, mixed ? 0 : 1, &m, &ri64_usex);
        if ((rc = upload_table(e, e->d_ri64, e->h_ri64))) {
            *rc_out = rc;
            return -1;
        }
        launch_residual_init<double>(e->d_ri64, grid_for(T, 2048), (int)ri64.size(), m, e->stream);
        for (int s : ri64) e->slots[s].outer_residuals++;
    }
    if (!sc.empty()) {
        unsigned m;
        int64_t T = fill_table(e, e->h_sc64, sc, false, 0, 0, nullptr);
        fill_table(e, e->h_sc32, sc, true, 0, 1, &m);
        if ((rc = upload_table(e, e->d_sc64, e->h_sc64)) || (rc = upload_table(e, e->d_sc32, e->h_sc32))) {
            *rc_out = rc;
            return -1;
        }
        launch_ir_scale(e->d_sc64, e->d_sc32, grid_for(T, 2048), e->stream);
        launch_residual_init<float>(e->d_sc32, grid_for(T, 2048), (int)sc.size(), m, e->stream);
    }
    // 2. iterations of every iterating slot
    std::vector<int> iter_ids;
    int64_t budget = INT64_MAX;
    for (int s = 0; s < e->max_slots; ++s) {
        Slot &sl = e->slots[s];
        if (sl.ph == S_ITER || sl.ph == S_INNER) {
            iter_ids.push_back(s);
            budget = std::min(budget, sl.max_iter - slot_max_iters(sl));
        }
    }
    std::stable_sort(iter_ids.begin(), iter_ids.end(),
                     [&](int a, int b) { return e->slots[a].kp < e->slots[b].kp; });
    if (iter_ids != e->main_ids) {
        // a system entering the table (first time, or back from a residual
        // check) starts at parity 0 on the next launch: its state was just
        // written to slot 1 by the residual kernel
        for (int sid : iter_ids)
            if (std::find(e->main_ids.begin(), e->main_ids.end(), sid) == e->main_ids.end())
                e->slots[sid].par_off = (int)(e->it_global & 1);
        e->main_ids = iter_ids;  // also when empty: a later return is an entry
        e->main_dirty = true;
    }
    // systems whose whole loop fits one workgroup run in k_solve_small; the
    // rest in the phase kernels of the main table (graph of m iterations)
    std::vector<int> big_ids, small_ids;
    for (int sid : iter_ids) (e->slots[sid].w->small ? small_ids : big_ids).push_back(sid);
    int nrun = 0;
    if (!iter_ids.empty()) {
        // small systems alone: the kernel iterates to convergence (or the
        // budget) in one launch; mixed with large ones, m at a time
        nrun = (int)std::max<int64_t>(1, std::min<int64_t>(budget, big_ids.empty() ? INT32_MAX : e->m));
        const bool dirty = e->main_dirty;
        if (!small_ids.empty()) {
            if (dirty) {
                fill_small_table(e, e->h_small, small_ids, mixed);
                if ((rc = upload_table(e, e->d_small, e->h_small))) {
                    *rc_out = rc;
                    return -1;
                }
            }
            if (mixed)
                launch_small<float>(e->d_small, e->small_count, e->small_res, (int)(e->it_global & 1), nrun,
                                    e->stream);
            else
                launch_small<double>(e->d_small, e->small_count, e->small_res, (int)(e->it_global & 1), nrun,
                                     e->stream);
            HIPCHK(hipGetLastError());
        }
        if (!big_ids.empty()) {
            int64_t T = 0;
            if (dirty) {
                T = fill_table(e, e->h_main, big_ids, mixed, 0, 0, &e->main_mask);
                if ((rc = upload_table(e, e->d_main, e->h_main))) {
                    *rc_out = rc;
                    return -1;
                }
            } else {
                T = e->h_main->total_tiles;
            }
            int cap = 1;
            for (int id : big_ids) cap = std::max(cap, grid_cap(e->slots[id].A, e->slots[id].w));
            const int grid = e->grid > 0 ? e->grid : grid_for(T, cap);
            if (e->use_graph && nrun == e->m) {
                if ((rc = ensure_graph(e, grid))) {
                    *rc_out = rc;
                    return -1;
                }
                hipError_t le = hipGraphLaunch(e->gexec[e->it_global & 1], e->stream);
                if (le != hipSuccess) {
                    *rc_out = fail(FEMCG_EDEVICE, "hipGraphLaunch: %s", hipGetErrorString(le));
                    return -1;
                }
                e->replays++;
            } else if ((rc = launch_iterations(e, nrun, grid, e->it_global))) {
                *rc_out = rc;
                return -1;
            }
        }
        e->main_dirty = false;
        e->it_global += nrun;
    }
    // 3. poll the states
    int hi = 0;
    for (int s = 0; s < e->max_slots; ++s)
        if (e->slots[s].ph != S_FREE && e->slots[s].ph != S_DONE) hi = s + 1;
    if (hi > 0) {
        hipError_t ce = hipMemcpyAsync(e->h_st64, e->d_st64, sizeof(SysState) * hi, hipMemcpyDeviceToHost, e->stream);
        if (ce == hipSuccess && mixed)
            ce = hipMemcpyAsync(e->h_st32, e->d_st32, sizeof(SysState) * hi, hipMemcpyDeviceToHost, e->stream);
        if (ce == hipSuccess) ce = hipStreamSynchronize(e->stream);
        if (ce != hipSuccess) {
            *rc_out = fail(FEMCG_EDEVICE, "state poll: %s", hipGetErrorString(ce));
            return -1;
        }
    }
    // 4. transitions
    int pending = 0;
    for (int s = 0; s < e->max_slots; ++s) {
        Slot &sl = e->slots[s];
        if (sl.ph == S_FREE || sl.ph == S_DONE) continue;
        const SysState &s64 = e->h_st64[s];
        const SysState &s32 = e->h_st32[s];
        auto finish = [&](int status) {
            sl.status = status;
            for (int j = 0; j < sl.k; ++j) sl.relres[j] = s64.relres[j];
            if (s64.status == FEMCG_EBREAKDOWN || (mixed && s32.status == FEMCG_EBREAKDOWN && status != FEMCG_OK))
                sl.status = FEMCG_EBREAKDOWN;
            sl.ph = S_DONE;
        };
        if (!mixed) {
            if (sl.ph == S_ITER) {
                for (int j = 0; j < sl.k; ++j) sl.iters[j] = s64.h_iters[j];
                sl.kernel_iters = slot_max_iters(sl);
            }
            switch (sl.ph) {
            case S_WAIT_START:
                if (s64.n_active == 0) finish(s64.status == FEMCG_EBREAKDOWN ? FEMCG_EBREAKDOWN : FEMCG_OK);
                else sl.ph = S_ITER;
                break;
            case S_ITER:
                if (s64.n_active == 0) {
                    sl.ph = S_CHECK;
                } else if (slot_max_iters(sl) >= sl.max_iter) {
                    sl.final_check = true;
                    sl.ph = S_CHECK;
                }
                break;
            case S_WAIT_CHECK:
                if (s64.n_active == 0) {
                    finish(FEMCG_OK);
                } else if (sl.final_check || sl.restarts >= sl.max_restarts) {
                    finish(FEMCG_WARN_MAXITER);
                } else {
                    sl.restarts++;
                    sl.ph = S_ITER;
                }
                break;
            default:
                break;
            }
        } else {
            switch (sl.ph) {
            case S_WAIT_START:
            case S_WAIT_OUTER:
                if (sl.ph == S_WAIT_OUTER) sl.outer++;
                if (s64.n_active == 0) finish(FEMCG_OK);
                else if (sl.outer >= sl.max_outer || slot_max_iters(sl) >= sl.max_iter)
                    finish(FEMCG_WARN_MAXITER);
                else sl.ph = S_OUTER;
                break;
            case S_WAIT_INNER:
                if (s32.n_active == 0) sl.ph = S_ACCUM;
                else sl.ph = S_INNER;
                break;
            case S_INNER: {
                int64_t inner_max = 0;
                for (int j = 0; j < sl.k; ++j) inner_max = std::max<int64_t>(inner_max, s32.h_iters[j]);
                if (s32.n_active == 0 || slot_max_iters(sl) + inner_max >= sl.max_iter) {
                    for (int j = 0; j < sl.k; ++j) sl.iters[j] += s32.h_iters[j];
                    sl.kernel_iters32 += inner_max;
                    sl.ph = S_ACCUM;
                }
                break;
            }
            default:
                break;
            }
        }
        if (sl.ph != S_DONE) ++pending;
    }
    return pending;
}

int require_device(const fem_matrix *A)
{
    if (A && A->host_only) return fail(FEMCG_EINVAL, "matrix assembled with FEM_ASSEMBLE_HOST_ONLY has no device copy");
    return FEMCG_OK;
}

int64_t default_max_iter(int64_t n)
{
    n = std::max<int64_t>(n, 2);
    return (int64_t)(20.0 * std::sqrt((double)n) * std::log2((double)n) + 100.0);
}

int upload_lifting(fem_matrix *A)
{
    const HostSystem &hs = A->hs;
    std::vector<int32_t> lr(hs.l_rowptr.begin(), hs.l_rowptr.end());
    int rc;
    if ((rc = upload(&A->d_lrow, lr))) return rc;
    if ((rc = upload(&A->d_lcol, hs.l_col))) return rc;
    if ((rc = upload(&A->d_lval, hs.l_val))) return rc;
    return FEMCG_OK;
}

void spmv_plan(const fem_matrix *A, int kp, Work &w)
{
    w.kp = kp;
    w.prec = PCG_FP64;
    w.n = A->dev.n;
    w.lpr = choose_lpr(A, kp);
    choose_tiles(A, kp, w.lpr, w.tile_rows, w.ntiles, w.band);
    w.ngroups = (w.ntiles + kGroup - 1) / kGroup;
}

SysDesc spmv_desc(const fem_matrix *A, const Work &w, int k, double *P, double *Q, double *part, double *gpart,
                  uint32_t *gticket, SysState *st)
{
    SysDesc D = make_desc_base(A, &w, false, nullptr, nullptr, nullptr, P, Q, part, st, k);
    D.band = w.band;
    D.lpr = w.lpr;
    D.gpart = gpart;
    D.gticket = gticket;
    D.tile_base = 0;
    return D;
}

int spmv_grid(const fem_matrix *A, const Work &w)
{
    return grid_for(w.ntiles, grid_cap(A, &w));
}

unsigned spmv_launch_mask(const Work &w)
{
    return launch_bit(w.kp, w.lpr);
}

}  // namespace femcg

using namespace femcg;

fem_matrix::~fem_matrix()
{
    engines.clear();
    works.clear();
    bcg.reset();
    free_dev(this);
    if (d_perm) (void)hipFree(d_perm);
    if (d_lrow) (void)hipFree(d_lrow);
    if (d_lcol) (void)hipFree(d_lcol);
    if (d_lval) (void)hipFree(d_lval);
}


// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
extern "C" {

const char *fem_last_error(void) { return g_err.c_str(); }

void pcg_default_opts(pcg_opts *o)
{
    if (!o) return;
    o->tol = 1e-8;
    o->max_iter = 0;
    o->precision = PCG_FP64;
    o->inner_eta = 1e-4;
    o->check_every = 32;
    o->use_x0 = 0;
    o->max_restarts = 3;
    o->max_outer = 30;
    o->use_graph = 1;
}

int fem_assemble(const fem_mesh *mesh, int32_t order, int32_t format, fem_matrix **out)
{
    g_err.clear();
    if (!mesh || !out) return fail(FEMCG_EINVAL, "NULL mesh or out");
    *out = nullptr;
    if ((format & FEM_ASSEMBLE_DEVICE) && (format & FEM_ASSEMBLE_HOST_ONLY))
        return fail(FEMCG_EINVAL, "FEM_ASSEMBLE_DEVICE and FEM_ASSEMBLE_HOST_ONLY exclude each other");
    const double t0 = now_s();
    auto A = std::make_unique<fem_matrix>();
    std::string err;
    int rc;
    try {
        rc = FEMCG_EUNSUPPORTED;
        if (format & FEM_ASSEMBLE_DEVICE) {
            rc = assemble_device(mesh, order, A->hs, err, nullptr);
            A->device_assembled = rc == FEMCG_OK;
        }
        if (rc == FEMCG_EUNSUPPORTED) {  // host assembly (also beyond the device path's ranges)
            A->hs = HostSystem{};
            err.clear();
            rc = assemble_host(mesh, order, A->hs, err);
        }
        if (rc) return fail(rc, "%s", err.c_str());
        if (A->hs.nfree == 0) return fail(FEMCG_EINVAL, "mesh has no free DOFs");
        const int fmt = (format & 0xf) == FEM_FORMAT_CSR ? FEM_FORMAT_CSR : FEM_FORMAT_SELL;
        const int sigma = (A->hs.order >= 2) ? 1024 : 1;
        rc = build_solver_copy(A->hs, fmt, 64, sigma, A->sc, err);
        if (rc) return fail(rc, "%s", err.c_str());
    } catch (const std::bad_alloc &) {
        return fail(FEMCG_ENOMEM, "host allocation failed during assembly");
    }
    A->host_only = (format & FEM_ASSEMBLE_HOST_ONLY) != 0;
    if (!A->host_only) {
        if ((rc = upload_solver_copy(A.get()))) return rc;
        if ((rc = upload_lifting(A.get()))) return rc;
    }
    if (const char *ev = std::getenv("FEMCG_MAX_GRID"))  // tuning override
        A->max_grid = std::max(kNumXcd, (atoi(ev) / kNumXcd) * kNumXcd);
    A->setup_s = now_s() - t0;
    A->stats.n = A->hs.nfree;
    A->stats.nnz = (int64_t)A->hs.a_col.size();
    A->stats.nnz_nonzero = A->sc.nnz;
    A->stats.nnz_stored = A->sc.stored;
    A->stats.setup_s = A->setup_s;
    A->stats.format = A->sc.format;
    *out = A.release();
    return FEMCG_OK;
}

void fem_free(fem_matrix *A) { delete A; }

static int fem_dofs_impl(const fem_matrix *A, int64_t *n_all, int64_t *n_free, double *dof_coords, uint8_t *dirichlet,
             int64_t *free2dof)
{
    if (!A) return fail(FEMCG_EINVAL, "NULL matrix");
    const HostSystem &hs = A->hs;
    if (n_all) *n_all = hs.ndofs;
    if (n_free) *n_free = hs.nfree;
    if (dof_coords) std::memcpy(dof_coords, hs.dof_coords.data(), sizeof(double) * hs.dof_coords.size());
    if (dirichlet) std::memcpy(dirichlet, hs.dirichlet.data(), hs.dirichlet.size());
    if (free2dof) std::memcpy(free2dof, hs.free2dof.data(), sizeof(int64_t) * hs.free2dof.size());
    return FEMCG_OK;
}

static int fem_csr_impl(const fem_matrix *A, int64_t *nnz, int64_t *rowptr, int32_t *col, double *val)
{
    if (!A) return fail(FEMCG_EINVAL, "NULL matrix");
    const HostSystem &hs = A->hs;
    if (nnz) *nnz = (int64_t)hs.a_col.size();
    if (rowptr) std::memcpy(rowptr, hs.a_rowptr.data(), sizeof(int64_t) * hs.a_rowptr.size());
    if (col) std::memcpy(col, hs.a_col.data(), sizeof(int32_t) * hs.a_col.size());
    if (val) std::memcpy(val, hs.a_val.data(), sizeof(double) * hs.a_val.size());
    return FEMCG_OK;
}

static int fem_rhs_impl(const fem_matrix *A, const double *g_all, int32_t k, double *B, void *stream)
{
    if (!A || !g_all || !B) return fail(FEMCG_EINVAL, "NULL argument");
    if (int rc = require_device(A)) return rc;
    if (k < 1 || k > kMaxK) return fail(FEMCG_EUNSUPPORTED, "k=%d outside 1..%d", k, kMaxK);
    const HostSystem &hs = A->hs;
    hipStream_t s = (hipStream_t)stream;
    std::vector<double> gd((size_t)std::max<int64_t>(hs.ndir, 1) * k, 0.0);
    for (int64_t i = 0; i < hs.ndir; ++i)
        std::memcpy(&gd[i * k], g_all + hs.dir2dof[i] * k, sizeof(double) * k);
    double *d_gd = nullptr;
    HIPCHK(hipMalloc((void **)&d_gd, sizeof(double) * gd.size()));
    HIPCHK(hipMemcpyAsync(d_gd, gd.data(), sizeof(double) * gd.size(), hipMemcpyHostToDevice, s));
    launch_lift(A->d_lrow, A->d_lcol, A->d_lval, d_gd, hs.nfree, k, B, s);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(s));
    HIPCHK(hipFree(d_gd));
    return FEMCG_OK;
}

static int fem_spmv_impl(fem_matrix *A, const double *X, double *Y, int32_t k, void *stream)
{
    if (!A || !X || !Y) return fail(FEMCG_EINVAL, "NULL argument");
    if (int rc = require_device(A)) return rc;
    if (k < 1 || k > kMaxK) return fail(FEMCG_EUNSUPPORTED, "k=%d outside 1..%d", k, kMaxK);
    hipStream_t s = (hipStream_t)stream;
    const int kp = pad_k(k);
    Work *w;
    int rc = get_work(A, kp, PCG_FP64, &w);
    if (rc) return rc;
    const int64_t n = A->dev.n;
    launch_gather(X, k, A->d_perm, n, k, kp, w->P64, s);
    // a private table and state: q = A p through the SpMM phase kernel
    SysTable *h = nullptr, *d = nullptr;
    SysState *st = nullptr;
    HIPCHK(hipHostMalloc((void **)&h, table_bytes(1), hipHostMallocDefault));
    HIPCHK(hipMalloc((void **)&d, table_bytes(1)));
    HIPCHK(hipMalloc((void **)&st, sizeof(SysState)));
    SysState hs0;
    init_state(hs0, k, kp, 1.0, 0.0);
    HIPCHK(hipMemcpyAsync(st, &hs0, sizeof hs0, hipMemcpyHostToDevice, s));
    SysDesc D = make_desc(A, w, false, w->B64, w->X64, w->R64, w->P64, w->Q64, w->part64, st, k);
    D.tile_base = 0;
    set_single_table(h, D);
    HIPCHK(hipMemcpyAsync(d, h, table_bytes(1), hipMemcpyHostToDevice, s));
    launch_phase<double>(PH_SPMM, d, grid_for(D.ntiles, grid_cap(A, w)), 0, 1, launch_bit(kp, w->lpr), s);
    launch_scatter(w->Q64, A->d_perm, n, k, kp, nullptr, Y, s);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(s));
    (void)hipHostFree(h);
    (void)hipFree(d);
    (void)hipFree(st);
    return FEMCG_OK;
}

static void fill_stats(fem_matrix *A, const Slot &sl, int prec, double solve_s, int64_t replays)
{
    pcg_stats_t &st = A->stats;
    st.n = A->hs.nfree;
    st.nnz = (int64_t)A->hs.a_col.size();
    st.nnz_nonzero = A->sc.nnz;
    st.nnz_stored = A->sc.stored;
    st.k = sl.k;
    st.status = sl.status;
    st.precision = prec;
    st.format = A->sc.format;
    st.outer = prec == PCG_MIXED ? sl.outer : sl.restarts + 1;
    st.graph_replays = (int32_t)replays;
    for (int j = 0; j < kMaxK; ++j) {
        st.iters[j] = j < sl.k ? sl.iters[j] : 0;
        st.relres[j] = j < sl.k ? sl.relres[j] : 0.0;
    }
    st.setup_s = A->setup_s;
    st.solve_s = solve_s;
    // algorithmic bytes per iteration: nnz*(s_v+4) + index array + 11 n k s_x + 2 n s_v
    const double n = (double)st.n, nnz = (double)st.nnz_nonzero, k = sl.k;
    auto it_bytes = [&](double sv) { return nnz * (sv + 4) + 4.0 * (n + 1) + 10.0 * n * k * sv + 2.0 * n * sv; };
    auto it_flops = [&]() { return 2.0 * nnz * k + 12.0 * n * k; };
    double bytes = 0, flops = 0;
    if (prec == PCG_FP64) {
        bytes = sl.kernel_iters * it_bytes(8.0);
        flops = sl.kernel_iters * it_flops();
    } else {
        bytes = sl.kernel_iters32 * it_bytes(4.0);
        flops = sl.kernel_iters32 * it_flops();
    }
    // residual evaluations: one SpMM + b, x read, r written
    bytes += sl.outer_residuals * (nnz * 12.0 + 4.0 * (n + 1) + 3.0 * n * k * 8.0);
    flops += sl.outer_residuals * 2.0 * nnz * k;
    st.bytes = bytes;
    st.gbps = solve_s > 0 ? bytes / solve_s / 1e9 : 0.0;
    st.gflops = solve_s > 0 ? flops / solve_s / 1e9 : 0.0;
    size_t fp = A->dev.bytes;
    for (auto &kv : A->works) fp += kv.second->bytes;
    st.footprint_mb = fp / 1e6;
}

static int get_engine(fem_matrix *A, int kp, int prec, int m, bool graph, Engine **out)
{
    auto key = std::make_pair(kp, prec);
    auto it = A->engines.find(key);
    if (it == A->engines.end()) {
        std::unique_ptr<Engine> e;
        int rc = engine_create(prec, 1, m, graph, e);
        if (rc) return rc;
        it = A->engines.emplace(key, std::move(e)).first;
    }
    Engine *e = it->second.get();
    e->m = std::max(1, m);
    e->use_graph = graph;
    *out = e;
    return FEMCG_OK;
}

static int pcg_solve_impl(fem_matrix *A, const double *B, double *X, int32_t k, double tol, const pcg_opts *opts_in,
              void *stream)
{
    g_err.clear();
    if (!A || !B || !X) return fail(FEMCG_EINVAL, "NULL argument");
    if (int rc = require_device(A)) return rc;
    if (k < 1 || k > kMaxK) return fail(FEMCG_EUNSUPPORTED, "k=%d outside 1..%d", k, kMaxK);
    pcg_opts o;
    pcg_default_opts(&o);
    if (opts_in) o = *opts_in;
    else o.tol = tol;
    if (!(o.tol > 0.0)) return fail(FEMCG_EINVAL, "tol must be > 0");
    if (o.precision != PCG_FP64 && o.precision != PCG_MIXED) return fail(FEMCG_EINVAL, "bad precision");
    const double t0 = now_s();
    hipStream_t s = (hipStream_t)stream;
    const int kp = pad_k(k);
    Work *w;
    int rc = get_work(A, kp, o.precision, &w);
    if (rc) return rc;
    Engine *e;
    if ((rc = get_engine(A, kp, o.precision, o.check_every > 0 ? o.check_every : 32, o.use_graph != 0, &e)))
        return rc;
    e->stream = s;
    e->grid = 0;
    Slot &sl = e->slots[0];
    sl = Slot{};
    sl.A = A;
    sl.w = w;
    sl.k = k;
    sl.kp = kp;
    sl.tol = o.tol;
    sl.max_iter = o.max_iter > 0 ? o.max_iter : default_max_iter(A->hs.nfree);
    sl.use_x0 = o.use_x0 ? 1 : 0;
    sl.max_restarts = std::max(0, o.max_restarts);
    sl.max_outer = std::max(1, o.max_outer);
    sl.eta = o.inner_eta > 0 ? o.inner_eta : 1e-4;
    const int64_t n = A->dev.n;
    launch_gather(B, k, A->d_perm, n, k, kp, w->B64, s);
    if (sl.use_x0) launch_gather(X, k, A->d_perm, n, k, kp, w->X64, s);
    HIPCHK(hipGetLastError());
    if ((rc = engine_admit(e, 0))) return rc;
    const int64_t replays0 = e->replays;
    int pending = 1;
    while (pending > 0) {
        pending = engine_tick(e, &rc);
        if (pending < 0) return rc;
    }
    launch_scatter(w->X64, A->d_perm, n, k, kp, e->d_st64, X, s);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(s));
    sl.ph = S_FREE;
    fill_stats(A, sl, o.precision, now_s() - t0, e->replays - replays0);
    A->last_kp = kp;
    A->last_prec = o.precision;
    if (sl.status == FEMCG_EBREAKDOWN) return fail(FEMCG_EBREAKDOWN, "breakdown: p.Ap <= 0 or non-finite scalar");
    return sl.status;
}

static int pcg_solve_batch_impl(int32_t nsys, fem_matrix *const *A, const double *const *B, double *const *X,
                    const int32_t *k, const double *tol, const pcg_opts *opts_in, int32_t *status, void *stream)
{
    g_err.clear();
    if (nsys < 1 || nsys > kMaxSys || !A || !B || !X || !k || !tol || !status)
        return fail(FEMCG_EINVAL, "bad batch arguments");
    pcg_opts o;
    pcg_default_opts(&o);
    if (opts_in) o = *opts_in;
    hipStream_t s = (hipStream_t)stream;
    const double t0 = now_s();
    for (int i = 0; i < nsys; ++i) {
        if (!A[i] || !B[i] || !X[i]) return fail(FEMCG_EINVAL, "NULL entry %d", i);
        if (int rc = require_device(A[i])) return rc;
        if (k[i] < 1 || k[i] > kMaxK) return fail(FEMCG_EUNSUPPORTED, "k[%d]=%d", i, k[i]);
        for (int j = 0; j < i; ++j)
            if (A[j] == A[i] && pad_k(k[j]) == pad_k(k[i]))
                return fail(FEMCG_EINVAL, "systems %d and %d share a matrix workspace", j, i);
    }
    std::unique_ptr<Engine> e;
    int rc = engine_create(o.precision, nsys, o.check_every > 0 ? o.check_every : 32, o.use_graph != 0, e);
    if (rc) return rc;
    e->stream = s;
    e->grid = A[0]->max_grid;
    int64_t tiles = 0;
    int cap = 1;
    for (int i = 0; i < nsys; ++i) {
        const int kp = pad_k(k[i]);
        Work *w;
        if ((rc = get_work(A[i], kp, o.precision, &w))) return rc;
        tiles += w->ntiles;
        cap = std::max(cap, grid_cap(A[i], w));
        Slot &sl = e->slots[i];
        sl = Slot{};
        sl.A = A[i];
        sl.w = w;
        sl.k = k[i];
        sl.kp = kp;
        sl.tol = tol[i];
        sl.max_iter = o.max_iter > 0 ? o.max_iter : default_max_iter(A[i]->hs.nfree);
        sl.use_x0 = o.use_x0 ? 1 : 0;
        sl.max_restarts = std::max(0, o.max_restarts);
        sl.max_outer = std::max(1, o.max_outer);
        sl.eta = o.inner_eta > 0 ? o.inner_eta : 1e-4;
        const int64_t n = A[i]->dev.n;
        launch_gather(B[i], k[i], A[i]->d_perm, n, k[i], kp, w->B64, s);
        if (sl.use_x0) launch_gather(X[i], k[i], A[i]->d_perm, n, k[i], kp, w->X64, s);
        if ((rc = engine_admit(e.get(), i))) return rc;
    }
    e->grid = grid_for(tiles, cap);
    int pending = nsys;
    while (pending > 0) {
        pending = engine_tick(e.get(), &rc);
        if (pending < 0) return rc;
    }
    int worst = 0;
    for (int i = 0; i < nsys; ++i) {
        Slot &sl = e->slots[i];
        launch_scatter(sl.w->X64, A[i]->d_perm, A[i]->dev.n, k[i], sl.kp, e->d_st64 + i, X[i], s);
        status[i] = sl.status;
        if (sl.status < 0) worst = sl.status;
        else if (sl.status > 0 && worst == 0) worst = sl.status;
    }
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(s));
    const double dt = now_s() - t0;
    for (int i = 0; i < nsys; ++i) fill_stats(A[i], e->slots[i], o.precision, dt, e->replays);
    return worst;
}

static int pcg_stats_impl(const fem_matrix *A, pcg_stats_t *out)
{
    if (!A || !out) return fail(FEMCG_EINVAL, "NULL argument");
    *out = A->stats;
    return FEMCG_OK;
}

static int fem_set_format_impl(fem_matrix *A, int32_t format_flags, int32_t C, int32_t sigma)
{
    if (!A) return fail(FEMCG_EINVAL, "NULL matrix");
    if (int rc = require_device(A)) return rc;
    const int sfc = (format_flags & FEM_ORDER_SFC) ? 1 : 0;
    const int format = format_flags & ~FEM_ORDER_SFC;
    if (format != FEM_FORMAT_CSR && format != FEM_FORMAT_SELL) return fail(FEMCG_EUNSUPPORTED, "format %d", format);
    if (format == FEM_FORMAT_SELL && (C < 1 || C > 64 || (C & (C - 1)))) return fail(FEMCG_EINVAL, "C=%d", C);
    std::string err;
    int rc = build_solver_copy(A->hs, format, format == FEM_FORMAT_SELL ? C : 64, std::max(1, sigma), A->sc, err, sfc);
    if (rc) return fail(rc, "%s", err.c_str());
    return upload_solver_copy(A);
}

// One SpMM launch on a matrix's own workspace, p zero-filled (values do not
// change the memory traffic), every tile forced: the timing probe of the
// autotuner and of the cold-cache measurement.
struct SpmmProbe {
    SysTable *h = nullptr, *d = nullptr;
    SysState *st = nullptr;
    int grid = 1;
    unsigned cm = 0;
    bool fp32 = false;
    int init(fem_matrix *A, int k, int precision, hipStream_t s)
    {
        const int kp = pad_k(k);
        Work *w;
        int rc = get_work(A, kp, precision, &w);
        if (rc) return rc;
        fp32 = precision == PCG_MIXED;
        void *P = fp32 ? (void *)w->P32 : (void *)w->P64;
        HIPCHK(hipMemsetAsync(P, 0, (size_t)A->dev.n * kp * (fp32 ? 4 : 8), s));
        HIPCHK(hipHostMalloc((void **)&h, table_bytes(1), hipHostMallocDefault));
        HIPCHK(hipMalloc((void **)&d, table_bytes(1)));
        HIPCHK(hipMalloc((void **)&st, sizeof(SysState)));
        HIPCHK(hipMemsetAsync(st, 0, sizeof(SysState), s));
        SysDesc D = fp32 ? make_desc(A, w, true, w->B32, w->X32, w->R32, w->P32, w->Q32, w->part32, st, k)
                         : make_desc(A, w, false, w->B64, w->X64, w->R64, w->P64, w->Q64, w->part64, st, k);
        D.tile_base = 0;
        set_single_table(h, D);
        HIPCHK(hipMemcpyAsync(d, h, table_bytes(1), hipMemcpyHostToDevice, s));
        HIPCHK(hipStreamSynchronize(s));
        cm = launch_bit(kp, w->lpr);
        grid = grid_for(D.ntiles, grid_cap(A, w));
        return FEMCG_OK;
    }
    void launch(hipStream_t s) const
    {
        if (fp32) launch_phase<float>(PH_SPMM, d, grid, 0, 1, cm, s);
        else launch_phase<double>(PH_SPMM, d, grid, 0, 1, cm, s);
    }
    ~SpmmProbe()
    {
        if (h) (void)hipHostFree(h);
        if (d) (void)hipFree(d);
        if (st) (void)hipFree(st);
    }
};

// Total time of `reps` calls of fn, bracketed by events on stream s.
static int time_launches(hipStream_t s, int reps, const std::function<void()> &fn, float *ms)
{
    hipEvent_t a, b;
    HIPCHK(hipEventCreate(&a));
    HIPCHK(hipEventCreate(&b));
    HIPCHK(hipEventRecord(a, s));
    for (int r = 0; r < reps; ++r) fn();
    HIPCHK(hipEventRecord(b, s));
    HIPCHK(hipEventSynchronize(b));
    HIPCHK(hipGetLastError());
    HIPCHK(hipEventElapsedTime(ms, a, b));
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    return FEMCG_OK;
}

// Autotuner: time the SpMM phase for each candidate layout on a synthetic p
// (the current solve data is irrelevant to its speed) and keep the fastest.
static int fem_tune_impl(fem_matrix *A, int32_t k, int32_t precision, int32_t *C_out, int32_t *sigma_out, void *stream)
{
    if (!A || k < 1 || k > kMaxK) return fail(FEMCG_EINVAL, "bad arguments");
    if (int rc = require_device(A)) return rc;
    if (precision != PCG_FP64 && precision != PCG_MIXED) return fail(FEMCG_EINVAL, "bad precision");
    hipStream_t s = (hipStream_t)stream;
    struct Cand {
        int format, C, sigma;
    };
    std::vector<Cand> cands = {{FEM_FORMAT_CSR, 64, 1}};
    for (int Cw : {16, 32, 64})
        for (int sg : {1, 64, 1024}) cands.push_back({FEM_FORMAT_SELL, Cw, sg});
    // 3D: the natural order puts face neighbours a whole plane of rows away;
    // P2: edge DOFs are numbered after all vertices, far from their
    // vertices' rows.  A Morton order keeps both near in index (and in cache)
    if (A->hs.dim == 3 || A->hs.order >= 2) {
        cands.push_back({FEM_FORMAT_CSR | FEM_ORDER_SFC, 64, 1});
        for (int Cw : {16, 32, 64}) cands.push_back({FEM_FORMAT_SELL | FEM_ORDER_SFC, Cw, 1});
    }
    const int kp = pad_k(k);
    double best = 1e30;
    Cand bc = cands[0];
    for (const Cand &c : cands) {
        int rc = fem_set_format(A, c.format, c.C, c.sigma);
        if (rc) return rc;
        SpmmProbe pr;
        if ((rc = pr.init(A, k, precision, s))) return rc;
        pr.launch(s);
        pr.launch(s);
        float t = 0;
        if ((rc = time_launches(s, 10, [&]() { pr.launch(s); }, &t))) return rc;
        if (t < best) {
            best = t;
            bc = c;
        }
    }
    int rc = fem_set_format(A, bc.format, bc.C, bc.sigma);
    if (rc) return rc;
    if (C_out) *C_out = bc.C;
    if (sigma_out) *sigma_out = bc.sigma;
    return bc.format;
}

static int fem_set_tiling_impl(fem_matrix *A, int32_t band, int32_t tile);

// Wall time of one pcg_solve on the caller's stream, from zero (X is
// overwritten); status of the solve in *status.
static int timed_solve(fem_matrix *A, const double *B, double *X, int k, const pcg_opts &o, hipStream_t s,
                       double *ms, int *status)
{
    HIPCHK(hipStreamSynchronize(s));
    const double t0 = now_s();
    *status = pcg_solve_impl(A, B, X, k, o.tol, &o, s);
    *ms = 1e3 * (now_s() - t0);
    return *status < 0 ? *status : FEMCG_OK;
}

static int pcg_tune_impl(fem_matrix *A, const double *B, int32_t k, double tol, pcg_opts *opts, pcg_tune_report *rep,
                         void *stream)
{
    g_err.clear();
    if (!A || !B || !opts || !rep) return fail(FEMCG_EINVAL, "NULL argument");
    if (int rc = require_device(A)) return rc;
    if (k < 1 || k > kMaxK) return fail(FEMCG_EUNSUPPORTED, "k=%d outside 1..%d", k, kMaxK);
    if (!(tol > 0.0)) return fail(FEMCG_EINVAL, "tol must be > 0");
    hipStream_t s = (hipStream_t)stream;
    pcg_tune_report R{};
    const int kp = pad_k(k);
    // 1. solver-copy format and row order (SpMM time)
    int32_t C = 0, sigma = 0;
    const int fmt = fem_tune_impl(A, k, PCG_FP64, &C, &sigma, stream);
    if (fmt < 0) return fmt;
    R.format = fmt & ~FEM_ORDER_SFC;
    R.sfc = (fmt & FEM_ORDER_SFC) ? 1 : 0;
    R.C = C;
    R.sigma = sigma;
    // 2. lanes per row of the one-column SpMM (SpMM time)
    A->lpr_force = 0;
    if (kp == 1) {
        float best = 1e30f;
        int bl = 1;
        for (int lpr : {1, 2, 4, 8}) {
            A->lpr_force = lpr;
            A->works.clear();
            A->engines.clear();
            SpmmProbe pr;
            int rc = pr.init(A, k, PCG_FP64, s);
            if (rc) return rc;
            pr.launch(s);
            pr.launch(s);
            float t = 0;
            if ((rc = time_launches(s, 10, [&]() { pr.launch(s); }, &t))) return rc;
            if (t < best) {
                best = t;
                bl = lpr;
            }
        }
        A->lpr_force = bl;
        A->works.clear();
        A->engines.clear();
    }
    R.lpr = choose_lpr(A, kp);
    double *X = nullptr;
    const size_t xbytes = sizeof(double) * (size_t)std::max<int64_t>(A->dev.n, 1) * k;
    if (hipMalloc((void **)&X, xbytes) != hipSuccess)
        return fail(FEMCG_ENOMEM, "tuner solution buffer of %zu bytes", xbytes);
    struct FreeOnExit {
        double *p;
        ~FreeOnExit() { (void)hipFree(p); }
    } free_x{X};
    pcg_opts o = *opts;
    o.tol = tol;
    o.use_x0 = 0;
    const int warm_iters = std::max(1, o.check_every > 0 ? o.check_every : 32);
    int rc, st;
    double ms;
    // 3. tiling of the phase kernels: the automatic tile, half and double,
    //    timed on capped FP64 solves, each after a warm-up solve that pays
    //    its graph capture
    Work *w;
    if ((rc = get_work(A, kp, PCG_FP64, &w))) return rc;
    R.band = w->small ? 2 : w->band;
    if (!w->small) {
        const int band = w->band;
        const int auto_tile = band ? w->tile_rows * kp * 8 : w->ntiles;
        std::vector<int> cands = {auto_tile};
        for (int t : {auto_tile / 2, auto_tile * 2})
            if (band ? (t >= 4096 && t <= 262144) : (t >= 64 && t <= 16384)) cands.push_back(t);
        pcg_opts oc = o;
        oc.precision = PCG_FP64;
        double best = 1e30;
        int bt = auto_tile;
        for (int t : cands) {
            if ((rc = fem_set_tiling_impl(A, band, t))) return rc;
            oc.max_iter = warm_iters;
            if ((rc = timed_solve(A, B, X, k, oc, s, &ms, &st))) return rc;
            oc.max_iter = 128;
            if ((rc = timed_solve(A, B, X, k, oc, s, &ms, &st))) return rc;
            if (ms < best) {
                best = ms;
                bt = t;
            }
        }
        if ((rc = fem_set_tiling_impl(A, band, bt))) return rc;
        R.tile = bt;
        if ((rc = get_work(A, kp, PCG_FP64, &w))) return rc;
    }
    R.ntiles = w->ntiles;
    // 4. precision and inner tolerance: full solves to tol, after a short
    //    warm-up solve of each precision (graph capture is not timed)
    pcg_opts o64 = o, omx = o;
    o64.precision = PCG_FP64;
    omx.precision = PCG_MIXED;
    {
        pcg_opts wu = o64;
        wu.max_iter = warm_iters;
        if ((rc = timed_solve(A, B, X, k, wu, s, &ms, &st))) return rc;
        wu.precision = PCG_MIXED;
        wu.max_outer = 1;
        if ((rc = timed_solve(A, B, X, k, wu, s, &ms, &st))) return rc;
    }
    if ((rc = timed_solve(A, B, X, k, o64, s, &R.fp64_ms, &st))) return rc;
    if (st != FEMCG_OK) return fail(FEMCG_EINVAL, "FP64 solve did not reach tol (status %d)", st);
    R.mixed_ms = 0.0;
    for (double eta : {1e-2, 1e-3, 1e-4, 1e-5}) {
        omx.inner_eta = eta;
        // a mixed solve that fails or misses tol is not a candidate
        if (timed_solve(A, B, X, k, omx, s, &ms, &st) == FEMCG_OK && st == FEMCG_OK &&
            (R.inner_eta == 0.0 || ms < R.mixed_ms)) {
            R.mixed_ms = ms;
            R.inner_eta = eta;
        }
    }
    g_err.clear();
    const bool mixed_wins = R.inner_eta > 0.0 && R.mixed_ms < R.fp64_ms;
    R.fp64_fallback = mixed_wins ? 0 : 1;
    R.precision = mixed_wins ? PCG_MIXED : PCG_FP64;
    *opts = o;
    opts->precision = R.precision;
    if (R.inner_eta > 0.0) opts->inner_eta = R.inner_eta;
    *rep = R;
    return FEMCG_OK;
}

static int fem_set_tiling_impl(fem_matrix *A, int32_t band, int32_t tile)
{
    if (!A || band < -1 || band > 2 || tile < 0) return fail(FEMCG_EINVAL, "bad tiling arguments");
    A->band_mode = band;
    if (band == 1) A->band_tile_bytes = tile > 0 ? std::max(1024, (int)tile) : 0;
    else A->tile_target = tile;
    A->engines.clear();
    A->works.clear();
    return FEMCG_OK;
}

static int pcg_time_kernel_impl(fem_matrix *A, int32_t kernel, int32_t reps, void *stream, double *ms, double *bytes)
{
    if (!A || !ms || kernel < 0 || kernel > 2 || reps < 1) return fail(FEMCG_EINVAL, "bad arguments");
    if (!A->last_kp) return fail(FEMCG_EINVAL, "no solve on this matrix yet");
    hipStream_t s = (hipStream_t)stream;
    const int kp = A->last_kp, prec = A->last_prec;
    Engine *e = A->engines[std::make_pair(kp, prec)].get();
    Work *w = A->works[std::make_pair(kp, prec)].get();
    if (!e || !w) return fail(FEMCG_EINVAL, "no workspace");
    const bool fp32 = prec == PCG_MIXED;
    // table of the last solve (slot 0), forced to run every tile
    SysTable *h = e->h_main;
    Slot &sl = e->slots[0];
    sl.A = A;
    sl.w = w;
    sl.k = A->stats.k;
    sl.kp = kp;
    std::vector<int> one{0};
    unsigned cm = 0;
    fill_table(e, h, one, fp32, 0, 0, &cm);
    HIPCHK(hipMemcpyAsync(e->d_main, h, table_bytes(1), hipMemcpyHostToDevice, s));
    e->main_ids.clear();
    e->main_dirty = true;
    const int grid = grid_for(h->total_tiles, grid_cap(A, w));
    auto launch = [&](int ph) {
        if (fp32) launch_phase<float>(ph, e->d_main, grid, 0, 1, cm, s);
        else launch_phase<double>(ph, e->d_main, grid, 0, 1, cm, s);
    };
    std::vector<hipEvent_t> ev(2 * (size_t)reps, nullptr);
    int rc = FEMCG_OK;
    for (auto &x : ev)
        if (hipEventCreate(&x) != hipSuccess) rc = fail(FEMCG_EDEVICE, "hipEventCreate failed");
    double tot = 0.0;
    if (rc == FEMCG_OK) {
        const int cls = (cm & kSplitBit) ? kSplitCls : class_of(kp);
        for (int ph = 0; ph < 3; ++ph) launch(ph);  // one untimed iteration
        for (int r = 0; r < reps; ++r)
            for (int ph = 0; ph < 3; ++ph) {
                if (ph != kernel) launch(ph);
                else if (fp32) launch_phase_timed<float>(ph, e->d_main, grid, 0, 1, cls, s, ev[2 * r], ev[2 * r + 1]);
                else launch_phase_timed<double>(ph, e->d_main, grid, 0, 1, cls, s, ev[2 * r], ev[2 * r + 1]);
            }
        hipError_t ce = hipEventSynchronize(ev[2 * reps - 1]);
        if (ce == hipSuccess) ce = hipGetLastError();
        if (ce != hipSuccess) rc = fail(FEMCG_EDEVICE, "kernel timing: %s", hipGetErrorString(ce));
        for (int r = 0; r < reps && rc == FEMCG_OK; ++r) {
            float t = 0;
            if (hipEventElapsedTime(&t, ev[2 * r], ev[2 * r + 1]) != hipSuccess)
                rc = fail(FEMCG_EDEVICE, "hipEventElapsedTime failed");
            tot += t;
        }
    }
    for (auto &x : ev)
        if (x) (void)hipEventDestroy(x);
    if (rc) return rc;
    *ms = tot / reps;
    if (bytes) {
        const double n = (double)A->sc.n, nnz = (double)A->sc.nnz, k = A->stats.k, sv = fp32 ? 4.0 : 8.0;
        const double idx = A->sc.format == FEM_FORMAT_SELL ? 4.0 * n : 4.0 * (n + 1);
        if (kernel == PH_SPMM) *bytes = nnz * (sv + 4.0) + idx + 2.0 * n * k * sv;
        else if (kernel == PH_UPDATE) *bytes = 3.0 * n * k * sv + n * sv;
        else *bytes = 5.0 * n * k * sv + n * sv;
    }
    return FEMCG_OK;
}

static int pcg_time_spmm_cold_impl(int32_t nmat, fem_matrix *const *A, int32_t k, int32_t precision, int32_t reps,
                       void *stream, double *ms, double *bytes)
{
    if (nmat < 1 || !A || !ms || k < 1 || k > kMaxK || reps < 1) return fail(FEMCG_EINVAL, "bad arguments");
    if (precision != PCG_FP64 && precision != PCG_MIXED) return fail(FEMCG_EINVAL, "bad precision");
    for (int i = 0; i < nmat; ++i)
        if (!A[i]) return fail(FEMCG_EINVAL, "NULL matrix %d", i);
        else if (int rc = require_device(A[i])) return rc;
    hipStream_t s = (hipStream_t)stream;
    std::vector<std::unique_ptr<SpmmProbe>> pr(nmat);
    int rc;
    double by = 0.0;
    const double sv = precision == PCG_MIXED ? 4.0 : 8.0;
    for (int i = 0; i < nmat; ++i) {
        pr[i].reset(new SpmmProbe);
        if ((rc = pr[i]->init(A[i], k, precision, s))) return rc;
        const double n = (double)A[i]->sc.n, nnz = (double)A[i]->sc.nnz;
        const double idx = A[i]->sc.format == FEM_FORMAT_SELL ? 4.0 * n : 4.0 * (n + 1);
        by += nnz * (sv + 4.0) + idx + 2.0 * n * k * sv;
    }
    for (int i = 0; i < nmat; ++i) pr[i]->launch(s);  // warm: leaves only the last copies cached
    float t = 0;
    if ((rc = time_launches(s, reps, [&]() {
             for (int i = 0; i < nmat; ++i) pr[i]->launch(s);
         }, &t)))
        return rc;
    *ms = t / ((double)reps * nmat);
    if (bytes) *bytes = by / nmat;
    return FEMCG_OK;
}


// Entry points: no C++ exception crosses the C ABI (a failed host allocation
// becomes FEMCG_ENOMEM, anything else FEMCG_EDEVICE with its message).

int fem_dofs(const fem_matrix *A, int64_t *n_all, int64_t *n_free, double *dof_coords, uint8_t *dirichlet, int64_t *free2dof)
{
    try {
        return fem_dofs_impl(A, n_all, n_free, dof_coords, dirichlet, free2dof);
    } catch (const std::bad_alloc &) {
        return fail(FEMCG_ENOMEM, "fem_dofs: host allocation failed");
    } catch (const std::exception &ex) {
        return fail(FEMCG_EDEVICE, "fem_dofs: %s", ex.what());
    }
}

int fem_csr(const fem_matrix *A, int64_t *nnz, int64_t *rowptr, int32_t *col, double *val)
{
    try {
        return fem_csr_impl(A, nnz, rowptr, col, val);
    } catch (const std::bad_alloc &) {
        return fail(FEMCG_ENOMEM, "fem_csr: host allocation failed");
    } catch (const std::exception &ex) {
        return fail(FEMCG_EDEVICE, "fem_csr: %s", ex.what());
    }
}

int fem_rhs(const fem_matrix *A, const double *g_all, int32_t k, double *B, void *stream)
{
    try {
        return fem_rhs_impl(A, g_all, k, B, stream);
    } catch (const std::bad_alloc &) {
        return fail(FEMCG_ENOMEM, "fem_rhs: host allocation failed");
    } catch (const std::exception &ex) {
        return fail(FEMCG_EDEVICE, "fem_rhs: %s", ex.what());
    }
}

int fem_spmv(fem_matrix *A, const double *X, double *Y, int32_t k, void *stream)
{
    try {
        return fem_spmv_impl(A, X, Y, k, stream);
    } catch (const std::bad_alloc &) {
        return fail(FEMCG_ENOMEM, "fem_spmv: host allocation failed");
    } catch (const std::exception &ex) {
        return fail(FEMCG_EDEVICE, "fem_spmv: %s", ex.what());
    }
}

int pcg_solve(fem_matrix *A, const double *B, double *X, int32_t k, double tol, const pcg_opts *opts, void *stream)
{
    try {
        return pcg_solve_impl(A, B, X, k, tol, opts, stream);
    } catch (const std::bad_alloc &) {
        return fail(FEMCG_ENOMEM, "pcg_solve: host allocation failed");
    } catch (const std::exception &ex) {
        return fail(FEMCG_EDEVICE, "pcg_solve: %s", ex.what());
    }
}

int pcg_solve_batch(int32_t nsys, fem_matrix *const *A, const double *const *B, double *const *X, const int32_t *k, const double *tol, const pcg_opts *opts, int32_t *status, void *stream)
{
    try {
        return pcg_solve_batch_impl(nsys, A, B, X, k, tol, opts, status, stream);
    } catch (const std::bad_alloc &) {
        return fail(FEMCG_ENOMEM, "pcg_solve_batch: host allocation failed");
    } catch (const std::exception &ex) {
        return fail(FEMCG_EDEVICE, "pcg_solve_batch: %s", ex.what());
    }
}

int pcg_stats(const fem_matrix *A, pcg_stats_t *out)
{
    try {
        return pcg_stats_impl(A, out);
    } catch (const std::bad_alloc &) {
        return fail(FEMCG_ENOMEM, "pcg_stats: host allocation failed");
    } catch (const std::exception &ex) {
        return fail(FEMCG_EDEVICE, "pcg_stats: %s", ex.what());
    }
}

int fem_tune(fem_matrix *A, int32_t k, int32_t precision, int32_t *C_out, int32_t *sigma_out, void *stream)
{
    try {
        return fem_tune_impl(A, k, precision, C_out, sigma_out, stream);
    } catch (const std::bad_alloc &) {
        return fail(FEMCG_ENOMEM, "fem_tune: host allocation failed");
    } catch (const std::exception &ex) {
        return fail(FEMCG_EDEVICE, "fem_tune: %s", ex.what());
    }
}

int pcg_tune(fem_matrix *A, const double *B, int32_t k, double tol, pcg_opts *opts, pcg_tune_report *report,
             void *stream)
{
    try {
        return pcg_tune_impl(A, B, k, tol, opts, report, stream);
    } catch (const std::bad_alloc &) {
        return fail(FEMCG_ENOMEM, "pcg_tune: host allocation failed");
    } catch (const std::exception &ex) {
        return fail(FEMCG_EDEVICE, "pcg_tune: %s", ex.what());
    }
}

int fem_set_format(fem_matrix *A, int32_t format, int32_t C, int32_t sigma)
{
    try {
        return fem_set_format_impl(A, format, C, sigma);
    } catch (const std::bad_alloc &) {
        return fail(FEMCG_ENOMEM, "fem_set_format: host allocation failed");
    } catch (const std::exception &ex) {
        return fail(FEMCG_EDEVICE, "fem_set_format: %s", ex.what());
    }
}

int fem_set_tiling(fem_matrix *A, int32_t band, int32_t tile)
{
    try {
        return fem_set_tiling_impl(A, band, tile);
    } catch (const std::bad_alloc &) {
        return fail(FEMCG_ENOMEM, "fem_set_tiling: host allocation failed");
    } catch (const std::exception &ex) {
        return fail(FEMCG_EDEVICE, "fem_set_tiling: %s", ex.what());
    }
}

int pcg_time_kernel(fem_matrix *A, int32_t kernel, int32_t reps, void *stream, double *ms, double *bytes)
{
    try {
        return pcg_time_kernel_impl(A, kernel, reps, stream, ms, bytes);
    } catch (const std::bad_alloc &) {
        return fail(FEMCG_ENOMEM, "pcg_time_kernel: host allocation failed");
    } catch (const std::exception &ex) {
        return fail(FEMCG_EDEVICE, "pcg_time_kernel: %s", ex.what());
    }
}

int pcg_time_spmm_cold(int32_t nmat, fem_matrix *const *A, int32_t k, int32_t precision, int32_t reps, void *stream, double *ms, double *bytes)
{
    try {
        return pcg_time_spmm_cold_impl(nmat, A, k, precision, reps, stream, ms, bytes);
    } catch (const std::bad_alloc &) {
        return fail(FEMCG_ENOMEM, "pcg_time_spmm_cold: host allocation failed");
    } catch (const std::exception &ex) {
        return fail(FEMCG_EDEVICE, "pcg_time_spmm_cold: %s", ex.what());
    }
}

}  // extern "C"
