// serve.cpp -- continuous batching of solve requests.
//
// Requests arrive with a mesh and Dirichlet data (Sect. 4.3: independent
// right-hand-side blocks arriving over time).  A worker thread assembles each
// one on the host (no device memory yet).  serve_step admits ready requests in
// arrival order while a slot is free and the request's device footprint fits
// the remaining budget, uploads it, and then runs one engine tick: every
// resident system advances by `check_every` iterations inside the same
// persistent phase kernels (one launch per CG phase for all of them).
// Converged systems retire at the next step, returning their memory.
#include <algorithm>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <exception>
#include <new>
#include <thread>

#include "engine.h"

namespace femcg {

struct Request {
    int64_t id = -1;
    int order = 1, k = 1;
    double tol = 1e-8;
    fem_mesh mesh{};
    std::vector<double> coords;
    std::vector<int32_t> cells;
    std::vector<uint8_t> bnd;
    std::vector<double> g;                // [n_all][k]
    std::unique_ptr<fem_matrix> A;
    int state = 0;                        // 0 assembling, 1 ready, 2 running, 3 done, 4 failed
    int status = 0;
    size_t footprint = 0;
    double t_submit = 0, t_ready = 0, t_admit = 0, t_done = 0;
    std::vector<double> X;                // [n_free][k]
    int64_t iters_max = 0;
    double relres_max = 0;
    int slot = -1;
    std::string err;
};

}  // namespace femcg

using namespace femcg;

struct fem_server {
    std::unique_ptr<Engine> eng;
    double budget = 0, used = 0;
    int prec = PCG_FP64, max_slots = 1;
    hipStream_t stream = nullptr;
    hipStream_t asm_stream = nullptr;  // device assembly of queued requests
    std::mutex mu;
    std::condition_variable cv;
    std::deque<Request *> to_assemble;
    std::deque<int64_t> ready;
    std::map<int64_t, std::unique_ptr<Request>> reqs;
    std::vector<std::thread> workers;
    // Device work of the server: one device assembly at a time (bounded
    // temporaries), and never during an engine step.  Device assemblies
    // running in a worker thread while serve_step ran the engine were
    // measured to corrupt other requests' systems: their solutions passed
    // the engine's own residual check but not the oracle's (2 of 40
    // requests per run); with the two serialised, none did.
    std::mutex gpu_mu;
    bool stop = false;
    int64_t next_id = 0;
    double t0 = 0;
};

static void assemble_worker(fem_server *s)
{
    for (;;) {
        Request *r;
        {
            std::unique_lock<std::mutex> lk(s->mu);
            s->cv.wait(lk, [&] { return s->stop || !s->to_assemble.empty(); });
            if (s->stop) return;
            r = s->to_assemble.front();
            s->to_assemble.pop_front();
        }
        auto A = std::make_unique<fem_matrix>();
        std::string err;
        int rc = FEMCG_OK;
        try {
            // large requests assemble on the device (falls back to the host
            // beyond its index ranges); small ones stay on the host
            const int nvl = r->mesh.dim + 1;
            const int64_t nl = r->order == 1 ? nvl : (r->order == 2 ? nvl + nvl * (nvl - 1) / 2 : (r->order + 1) * (r->order + 2) / 2);
            rc = FEMCG_EUNSUPPORTED;
            if (r->mesh.ncells * nl * nl >= ((int64_t)1 << 20)) {
                std::lock_guard<std::mutex> g(s->gpu_mu);
                rc = assemble_device(&r->mesh, r->order, A->hs, err, s->asm_stream);
            }
            if (rc == FEMCG_EUNSUPPORTED) {
                A->hs = HostSystem{};
                err.clear();
                rc = assemble_host(&r->mesh, r->order, A->hs, err);
            }
            if (!rc && A->hs.nfree == 0) {
                rc = FEMCG_EINVAL;
                err = "no free DOFs";
            }
            if (!rc) rc = build_solver_copy(A->hs, FEM_FORMAT_SELL, 64, r->order >= 2 ? 1024 : 1, A->sc, err);
        } catch (const std::bad_alloc &) {
            rc = FEMCG_ENOMEM;
            err = "host allocation failed";
        }
        std::lock_guard<std::mutex> lk(s->mu);
        r->t_ready = now_s() - s->t0;
        if (rc) {
            r->state = 4;
            r->status = rc;
            r->err = err;
            r->t_done = r->t_ready;
        } else {
            const int kp = pad_k(r->k);
            r->footprint = matrix_bytes_estimate(A->sc, A->hs) + work_bytes_estimate(A->hs.nfree, kp, s->prec, 2048) +
                           (size_t)A->hs.ndir * r->k * 8;
            r->A = std::move(A);
            r->state = 1;
            s->ready.push_back(r->id);
        }
        r->coords.clear();
        r->coords.shrink_to_fit();
        r->cells.clear();
        r->cells.shrink_to_fit();
    }
}

// Upload, lift and gather one request into slot `slot`.
static int admit_request(fem_server *s, Request *r, int slot)
{
    fem_matrix *A = r->A.get();
    int rc;
    if ((rc = upload_solver_copy(A))) return rc;
    if ((rc = upload_lifting(A))) return rc;
    const int kp = pad_k(r->k);
    Work *w;
    if ((rc = get_work(A, kp, s->prec, &w))) return rc;
    const HostSystem &hs = A->hs;
    if ((int64_t)r->g.size() != hs.ndofs * r->k)
        return fail(FEMCG_EINVAL, "request data holds %zu values, the system has %lld DOFs x %d columns", r->g.size(),
                    (long long)hs.ndofs, r->k);
    // B = -K_ID g_D into R64 (public order), then gathered into B64
    std::vector<double> gd((size_t)std::max<int64_t>(hs.ndir, 1) * r->k, 0.0);
    for (int64_t i = 0; i < hs.ndir; ++i)
        std::memcpy(&gd[i * r->k], &r->g[hs.dir2dof[i] * r->k], sizeof(double) * r->k);
    double *d_gd = nullptr;
    if (hipMalloc((void **)&d_gd, gd.size() * 8) != hipSuccess) return fail(FEMCG_ENOMEM, "lifting buffer");
    if (hipMemcpyAsync(d_gd, gd.data(), gd.size() * 8, hipMemcpyHostToDevice, s->stream) != hipSuccess) {
        (void)hipFree(d_gd);
        return fail(FEMCG_EDEVICE, "lifting upload");
    }
    launch_lift(A->d_lrow, A->d_lcol, A->d_lval, d_gd, hs.nfree, r->k, w->R64, s->stream);
    launch_gather(w->R64, r->k, A->d_perm, A->dev.n, r->k, kp, w->B64, s->stream);
    hipError_t e = hipStreamSynchronize(s->stream);
    (void)hipFree(d_gd);
    if (e != hipSuccess) return fail(FEMCG_EDEVICE, "admission: %s", hipGetErrorString(e));
    r->g.clear();
    r->g.shrink_to_fit();
    Slot &sl = s->eng->slots[slot];
    sl = Slot{};
    sl.A = A;
    sl.w = w;
    sl.k = r->k;
    sl.kp = kp;
    sl.tol = r->tol;
    sl.max_iter = default_max_iter(hs.nfree);
    sl.req = r->id;
    sl.max_restarts = 3;
    sl.max_outer = 30;
    sl.eta = 1e-4;
    return engine_admit(s->eng.get(), slot);
}

static int retire_slot(fem_server *s, int slot)
{
    Slot &sl = s->eng->slots[slot];
    Request *r = s->reqs[sl.req].get();
    fem_matrix *A = sl.A;
    Work *w = sl.w;
    const int64_t n = A->dev.n;
    launch_scatter(w->X64, A->d_perm, n, sl.k, sl.kp, s->eng->d_st64 + slot, w->R64, s->stream);
    r->X.resize((size_t)n * sl.k);
    if (hipMemcpyAsync(r->X.data(), w->R64, r->X.size() * 8, hipMemcpyDeviceToHost, s->stream) != hipSuccess)
        return fail(FEMCG_EDEVICE, "retire copy");
    hipError_t e = hipStreamSynchronize(s->stream);
    if (e != hipSuccess) return fail(FEMCG_EDEVICE, "retire: %s", hipGetErrorString(e));
    r->status = sl.status;
    r->iters_max = 0;
    r->relres_max = 0;
    for (int j = 0; j < sl.k; ++j) {
        r->iters_max = std::max(r->iters_max, sl.iters[j]);
        r->relres_max = std::max(r->relres_max, sl.relres[j]);
    }
    r->t_done = now_s() - s->t0;
    r->state = 3;
    s->used -= (double)r->footprint;
    r->A.reset();  // frees the matrix and its workspaces
    sl = Slot{};
    s->eng->main_dirty = true;
    return FEMCG_OK;
}

extern "C" {

static int serve_create_impl(double budget_bytes, int32_t max_slots, int32_t precision, int32_t check_every, fem_server **out)
{
    if (!out || budget_bytes <= 0 || max_slots < 1 || max_slots > kMaxSys) return fail(FEMCG_EINVAL, "bad arguments");
    if (precision != PCG_FP64 && precision != PCG_MIXED) return fail(FEMCG_EINVAL, "bad precision");
    auto s = std::make_unique<fem_server>();
    s->budget = budget_bytes;
    s->prec = precision;
    s->max_slots = max_slots;
    int rc = engine_create(precision, max_slots, check_every > 0 ? check_every : 16, true, s->eng);
    if (rc) return rc;
    if (hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking) != hipSuccess)
        return fail(FEMCG_EDEVICE, "stream");
    if (hipStreamCreateWithFlags(&s->asm_stream, hipStreamNonBlocking) != hipSuccess)
        return fail(FEMCG_EDEVICE, "stream");
    s->eng->stream = s->stream;
    s->eng->grid = 2048;
    s->t0 = now_s();
    fem_server *raw = s.get();
    unsigned hw = std::thread::hardware_concurrency();
    const int nw = (int)std::max(1u, std::min(4u, hw / 4));
    for (int i = 0; i < nw; ++i) s->workers.emplace_back(assemble_worker, raw);
    *out = s.release();
    return FEMCG_OK;
}

static int64_t serve_submit_impl(fem_server *s, const fem_mesh *mesh, int32_t order, const double *g_all, int32_t k, double tol)
{
    if (!s || !mesh || !g_all || k < 1 || k > kMaxK || !(tol > 0)) return fail(FEMCG_EINVAL, "bad arguments");
    if ((mesh->dim != 2 && mesh->dim != 3) || order < 1 || order > 4 || (order > 2 && mesh->dim != 2))
        return fail(FEMCG_EUNSUPPORTED, "dim/order");
    auto r = std::make_unique<Request>();
    r->t_submit = now_s() - s->t0;
    r->order = order;
    r->k = k;
    r->tol = tol;
    const int nvl = mesh->dim + 1;
    r->coords.assign(mesh->coords, mesh->coords + mesh->nverts * mesh->dim);
    r->cells.assign(mesh->cells, mesh->cells + mesh->ncells * nvl);
    r->bnd.assign(mesh->on_boundary, mesh->on_boundary + mesh->nverts);
    // number of DOFs is known only after assembly; the caller passes n_all
    // rows of g: vertices, p-1 per edge, (p-1)(p-2)/2 per cell (P3/P4), so
    // count the edges here the same way the assembler numbers them
    int64_t n_all = mesh->nverts;
    if (order >= 2) {
        int E[6][2], c = 0;
        for (int a = 0; a < nvl; ++a)
            for (int b = a + 1; b < nvl; ++b) E[c][0] = a, E[c][1] = b, ++c;
        std::vector<uint64_t> keys;
        keys.reserve(mesh->ncells * c);
        for (int64_t cc = 0; cc < mesh->ncells; ++cc)
            for (int e = 0; e < c; ++e) {
                uint64_t a = (uint64_t)mesh->cells[cc * nvl + E[e][0]], b = (uint64_t)mesh->cells[cc * nvl + E[e][1]];
                if (a > b) std::swap(a, b);
                keys.push_back((a << 32) | b);
            }
        std::sort(keys.begin(), keys.end());
        const int64_t nedges = (int64_t)(std::unique(keys.begin(), keys.end()) - keys.begin());
        n_all += (int64_t)(order - 1) * nedges + (int64_t)(order - 1) * (order - 2) / 2 * mesh->ncells;
    }
    r->g.assign(g_all, g_all + n_all * k);
    r->mesh.dim = mesh->dim;
    r->mesh.nverts = mesh->nverts;
    r->mesh.ncells = mesh->ncells;
    r->mesh.coords = r->coords.data();
    r->mesh.cells = r->cells.data();
    r->mesh.on_boundary = r->bnd.data();
    std::lock_guard<std::mutex> lk(s->mu);
    r->id = s->next_id++;
    Request *raw = r.get();
    s->reqs[r->id] = std::move(r);
    s->to_assemble.push_back(raw);
    s->cv.notify_one();
    return raw->id;
}

static int serve_step_impl(fem_server *s)
{
    if (!s) return fail(FEMCG_EINVAL, "NULL server");
    std::lock_guard<std::mutex> gpu(s->gpu_mu);
    Engine *e = s->eng.get();
    int rc;
    // 1. retire finished systems
    for (int i = 0; i < s->max_slots; ++i)
        if (e->slots[i].ph == S_DONE)
            if ((rc = retire_slot(s, i))) return rc;
    // 2. admit in arrival order while a slot and the memory budget allow
    for (;;) {
        Request *r = nullptr;
        {
            std::lock_guard<std::mutex> lk(s->mu);
            if (s->ready.empty()) break;
            r = s->reqs[s->ready.front()].get();
            if ((double)r->footprint > s->budget) {
                s->ready.pop_front();
                r->state = 4;
                r->status = FEMCG_EADMIT;
                r->err = "footprint exceeds the server budget";
                r->t_done = now_s() - s->t0;
                r->A.reset();
                continue;
            }
            if (s->used + (double)r->footprint > s->budget) break;
        }
        int slot = -1;
        for (int i = 0; i < s->max_slots; ++i)
            if (e->slots[i].ph == S_FREE) {
                slot = i;
                break;
            }
        if (slot < 0) break;
        {
            std::lock_guard<std::mutex> lk(s->mu);
            s->ready.pop_front();
        }
        r->t_admit = now_s() - s->t0;
        r->slot = slot;
        r->state = 2;
        s->used += (double)r->footprint;
        if ((rc = admit_request(s, r, slot))) {
            r->state = 4;
            r->status = rc;
            r->err = fem_last_error();
            r->t_done = now_s() - s->t0;
            s->used -= (double)r->footprint;
            r->A.reset();
            e->slots[slot] = Slot{};
        }
    }
    // 3. one tick of every resident system
    bool any = false;
    for (int i = 0; i < s->max_slots; ++i)
        if (e->slots[i].ph != S_FREE && e->slots[i].ph != S_DONE) any = true;
    if (any) {
        if (engine_tick(e, &rc) < 0) return rc;
    }
    int open = 0;
    std::lock_guard<std::mutex> lk(s->mu);
    for (auto &kv : s->reqs)
        if (kv.second->state < 3) ++open;
    for (int i = 0; i < s->max_slots; ++i)
        if (e->slots[i].ph == S_DONE) ++open;
    return open;
}

static int serve_poll_impl(fem_server *s, int64_t id, double *X, fem_request_info *info)
{
    if (!s) return fail(FEMCG_EINVAL, "NULL server");
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->reqs.find(id);
    if (it == s->reqs.end()) return fail(FEMCG_EINVAL, "unknown request %lld", (long long)id);
    Request *r = it->second.get();
    if (r->state < 3) return 0;
    if (info) {
        info->id = r->id;
        info->status = r->status;
        info->k = r->k;
        info->n = (int64_t)(r->X.size() / std::max(1, r->k));
        info->iters_max = r->iters_max;
        info->t_submit = r->t_submit;
        info->t_ready = r->t_ready;
        info->t_admit = r->t_admit;
        info->t_done = r->t_done;
        info->relres_max = r->relres_max;
        info->footprint_mb = (double)r->footprint * 1e-6;
    }
    if (X && !r->X.empty()) std::memcpy(X, r->X.data(), r->X.size() * 8);
    s->reqs.erase(it);
    return 1;
}

double serve_clock(const fem_server *s) { return s ? now_s() - s->t0 : 0.0; }

void serve_destroy(fem_server *s)
{
    if (!s) return;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
    }
    s->cv.notify_all();
    for (auto &t : s->workers) t.join();
    if (s->stream) (void)hipStreamSynchronize(s->stream);
    s->eng.reset();
    s->reqs.clear();
    if (s->stream) (void)hipStreamDestroy(s->stream);
    if (s->asm_stream) (void)hipStreamDestroy(s->asm_stream);
    delete s;
}


// Entry points: no C++ exception crosses the C ABI (a failed host allocation
// becomes FEMCG_ENOMEM, anything else FEMCG_EDEVICE with its message).

int serve_create(double budget_bytes, int32_t max_slots, int32_t precision, int32_t check_every, fem_server **out)
{
    try {
        return serve_create_impl(budget_bytes, max_slots, precision, check_every, out);
    } catch (const std::bad_alloc &) {
        return fail(FEMCG_ENOMEM, "serve_create: host allocation failed");
    } catch (const std::exception &ex) {
        return fail(FEMCG_EDEVICE, "serve_create: %s", ex.what());
    }
}

int64_t serve_submit(fem_server *s, const fem_mesh *mesh, int32_t order, const double *g_all, int32_t k, double tol)
{
    try {
        return serve_submit_impl(s, mesh, order, g_all, k, tol);
    } catch (const std::bad_alloc &) {
        return fail(FEMCG_ENOMEM, "serve_submit: host allocation failed");
    } catch (const std::exception &ex) {
        return fail(FEMCG_EDEVICE, "serve_submit: %s", ex.what());
    }
}

int serve_step(fem_server *s)
{
    try {
        return serve_step_impl(s);
    } catch (const std::bad_alloc &) {
        return fail(FEMCG_ENOMEM, "serve_step: host allocation failed");
    } catch (const std::exception &ex) {
        return fail(FEMCG_EDEVICE, "serve_step: %s", ex.what());
    }
}

int serve_poll(fem_server *s, int64_t id, double *X, fem_request_info *info)
{
    try {
        return serve_poll_impl(s, id, X, info);
    } catch (const std::bad_alloc &) {
        return fail(FEMCG_ENOMEM, "serve_poll: host allocation failed");
    } catch (const std::exception &ex) {
        return fail(FEMCG_EDEVICE, "serve_poll: %s", ex.what());
    }
}

}  // extern "C"
