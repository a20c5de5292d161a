// C ABI of the library (declared in include/hodlr.h): argument checks,
// handle lifetime, device-memory accounting and error reporting.  No
// exception crosses this boundary.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>

#include "hodlr_impl.hpp"

namespace {
thread_local std::string g_last_error;

hodlr_status set_error(hodlr_status c, const std::string& m) {
    g_last_error = m;
    return c;
}

template <typename F>
hodlr_status guarded(F&& f) {
    try {
        g_last_error.clear();
        f();
        return HODLR_OK;
    } catch (const hodlr::Error& e) {
        return set_error(e.code, e.msg);
    } catch (const std::bad_alloc&) {
        return set_error(HODLR_ENOMEM, "host allocation failed");
    } catch (...) {
        return set_error(HODLR_EDEVICE, "unexpected internal error");
    }
}

double ms_since(std::chrono::steady_clock::time_point t0) {
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
}

void free_all(hodlr_t h) {
    for (auto& kv : h->allocs) (void)hipFree(kv.first);
    h->allocs.clear();
    if (h->ev_fork) (void)hipEventDestroy(h->ev_fork);
    if (h->ev_join) (void)hipEventDestroy(h->ev_join);
    if (h->aux) (void)hipStreamDestroy(h->aux);
    h->ev_fork = h->ev_join = nullptr;
    h->aux = nullptr;
}
}  // namespace

namespace hodlr {

void* dalloc(hodlr_t h, size_t bytes) {
    bytes = std::max<size_t>(bytes, 16);
    if (h->opts.mem_budget_bytes && h->device_bytes + bytes > h->opts.mem_budget_bytes)
        fail(HODLR_ENOMEM, "device memory budget exceeded");
    void* p = nullptr;
    if (hipMalloc(&p, bytes) != hipSuccess || !p) {
        (void)hipGetLastError();
        fail(HODLR_ENOMEM, "device allocation of " + std::to_string(bytes) + " bytes failed");
    }
    h->allocs[p] = bytes;
    h->device_bytes += bytes;
    return p;
}

void dfree(hodlr_t h, void* p) {
    if (!p) return;
    auto it = h->allocs.find(p);
    if (it == h->allocs.end()) return;
    h->device_bytes -= it->second;
    h->allocs.erase(it);
    (void)hipFree(p);
}

}  // namespace hodlr

extern "C" {

void hodlr_default_opts(hodlr_opts* o) {
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->level_rule = 1;
    o->has_domain = 0;
    o->domain_side = 1.0;
    o->storage = HODLR_FP64;
    o->symmetric = 1;
    o->max_rank = 0;
    o->skip_aca = 0;
    o->mem_budget_bytes = 0;
    o->adm_dim = 0;
    o->skeleton = 0;
}

hodlr_status hodlr_build(const double* points, int64_t N, int d, const hodlr_kernel* kernel,
                         int leaf_size, double tol, const hodlr_opts* opts, void* stream,
                         hodlr_t* out) {
    if (!points || !kernel || !out) return set_error(HODLR_EINVAL, "null pointer argument");
    if (N < 1 || N > INT32_MAX) return set_error(HODLR_EINVAL, "N must be in [1, 2^31)");
    if (d < 1 || d > 8) return set_error(HODLR_EINVAL, "d must be in [1, 8]");
    if (leaf_size < 1) return set_error(HODLR_EINVAL, "leaf_size must be >= 1");
    if (!(tol >= 0.0 && tol < 1.0)) return set_error(HODLR_EINVAL, "tol must be in [0, 1)");
    if (kernel->kind < HODLR_K_LOG || kernel->kind > HODLR_K_INV_SQRT1P)
        return set_error(HODLR_EINVAL, "unknown kernel kind");
    if ((kernel->kind == HODLR_K_GAUSS || kernel->kind == HODLR_K_EXP) && !(kernel->h > 0.0))
        return set_error(HODLR_EINVAL, "kernel length scale h must be > 0");
    hodlr_opts o;
    hodlr_default_opts(&o);
    if (opts) o = *opts;
    if (o.level_rule < 0 || o.level_rule > 2) return set_error(HODLR_EINVAL, "bad level_rule");
    if (o.storage != HODLR_FP64 && o.storage != HODLR_FP32 && o.storage != HODLR_BF16)
        return set_error(HODLR_EINVAL, "storage must be FP64, FP32 or BF16");
    if (o.has_domain && !(o.domain_side > 0.0 && std::isfinite(o.domain_side)))
        return set_error(HODLR_EINVAL, "domain_side must be > 0");
    if (o.max_rank < 0) return set_error(HODLR_EINVAL, "max_rank must be >= 0");
    if (o.adm_dim < -1 || o.adm_dim > d - 1)
        return set_error(HODLR_EINVAL, "adm_dim must be in -1 .. d-1");
    if (o.skeleton != 0 && o.skeleton != 1) return set_error(HODLR_EINVAL, "skeleton must be 0 or 1");
    if (o.skeleton && o.storage != HODLR_FP64)
        return set_error(HODLR_EINVAL, "the skeleton form stores FP64 (its solves with "
                                       "K(sigma, tau) need the products to full precision)");
    if (o.skeleton && o.skip_aca)
        return set_error(HODLR_EINVAL, "the skeleton form takes its factors from ACA (skip_aca = 0)");

    hodlr_t h = new (std::nothrow) hodlr_handle_s();
    if (!h) return set_error(HODLR_ENOMEM, "host allocation failed");
    h->N = N;
    h->d = d;
    h->kern = *kernel;
    h->leaf = leaf_size;
    h->tol = tol;
    h->opts = o;
    h->kp.kind = kernel->kind;
    h->kp.h = kernel->h;
    h->kp.inv_h = kernel->h > 0 ? 1.0 / kernel->h : 0.0;
    h->kp.inv_h2 = kernel->h > 0 ? 1.0 / (kernel->h * kernel->h) : 0.0;
    h->kp.scale = kernel->scale;
    h->kp.diag = kernel->diag;
    hipStream_t s = (hipStream_t)stream;
    hodlr_status st = guarded([&] {
        HIP_CHECK(hipGetDevice(&h->device));
        auto t0 = std::chrono::steady_clock::now();
        hodlr::build_tree(h, points, s);
        h->build_ms[0] = ms_since(t0);
        t0 = std::chrono::steady_clock::now();
        hodlr::build_lists(h, s);
        hodlr::build_block_table(h, s);
        h->build_ms[1] = ms_since(t0);
        t0 = std::chrono::steady_clock::now();
        if (!o.skip_aca) {
            hodlr::compress_all(h, s);
        } else if (h->kappa == 0) {
            hodlr::finalize_factors(h, s);
        }
        h->build_ms[2] = ms_since(t0);
    });
    if (st != HODLR_OK) {
        (void)hipStreamSynchronize(s);
        free_all(h);
        delete h;
        return st;
    }
    *out = h;
    return HODLR_OK;
}

namespace {
hodlr_status matvec_checked(hodlr_t h, const void* X, int64_t ldx, int nrhs, int x_prec, void* Y,
                            int64_t ldy, int compute_prec, void* stream, void* const* events,
                            int nevents, bool noalloc = false) {
    if (!h || !X || !Y) return set_error(HODLR_EINVAL, "null pointer argument");
    if (nrhs < 1) return set_error(HODLR_EINVAL, "nrhs must be >= 1");
    if (ldx < h->N || ldy < h->N) return set_error(HODLR_EINVAL, "leading dimension < N");
    if (x_prec != HODLR_FP64 && x_prec != HODLR_FP32)
        return set_error(HODLR_EINVAL, "x_prec must be FP64 or FP32");
    if (compute_prec != HODLR_FP64 && compute_prec != HODLR_FP32)
        return set_error(HODLR_EINVAL, "compute_prec must be FP64 or FP32");
    if (h->opts.storage == HODLR_BF16 && compute_prec != HODLR_FP32)
        return set_error(HODLR_EINVAL, "BF16 factors are applied in FP32 arithmetic");
    if (h->opts.skeleton && compute_prec != HODLR_FP64)
        return set_error(HODLR_EINVAL, "the skeleton form is applied in FP64 arithmetic");
    if (events && nevents != 5 && nevents != 5 + hodlr::kApplyClasses)
        return set_error(HODLR_EINVAL, "events must hold 5 or 11 entries");
    for (int l = 1; l <= h->kappa; ++l)
        if (!h->lev[l].has_factors) return set_error(HODLR_EINVAL, "factors missing");
    if (!h->near_items) return set_error(HODLR_EINVAL, "factors missing");
    return guarded([&] {
        if (noalloc)
            hodlr::matvec_noalloc(h, X, ldx, nrhs, x_prec, Y, ldy, compute_prec,
                                  (hipStream_t)stream);
        else
            hodlr::matvec(h, X, ldx, nrhs, x_prec, Y, ldy, compute_prec,
                          reinterpret_cast<hipEvent_t const*>(events), events ? nevents : 0,
                          (hipStream_t)stream);
    });
}
}  // namespace

hodlr_status hodlr_reserve_workspace(hodlr_t h, int nrhs, int compute_prec) {
    if (!h) return set_error(HODLR_EINVAL, "null handle");
    if (nrhs < 1) return set_error(HODLR_EINVAL, "nrhs must be >= 1");
    if (compute_prec != HODLR_FP64 && compute_prec != HODLR_FP32)
        return set_error(HODLR_EINVAL, "compute_prec must be FP64 or FP32");
    return guarded([&] { hodlr::reserve_workspace(h, nrhs, compute_prec, nullptr); });
}

hodlr_status hodlr_mfma_extent(int64_t rank, int64_t len, int nrhs, int64_t* extent) {
    if (rank < 0 || len < 0 || nrhs < 1 || nrhs > 32 || !extent)
        return set_error(HODLR_EINVAL, "rank, len >= 0, 1 <= nrhs <= 32, extent non-null");
    const int nrp = nrhs <= 16 ? 16 : 32;
    *extent = hodlr::mcore_extent(rank, len, nrp);
    if (*extent >= hodlr::kMcoreRange)
        return set_error(HODLR_EUNSUPPORTED, "factor exceeds the matrix-core buffer range");
    return HODLR_OK;
}

hodlr_status hodlr_matvec(hodlr_t h, const void* X, int64_t ldx, int nrhs, int x_prec, void* Y,
                          int64_t ldy, int compute_prec, void* stream) {
    return matvec_checked(h, X, ldx, nrhs, x_prec, Y, ldy, compute_prec, stream, nullptr, 0);
}

hodlr_status hodlr_set_route(hodlr_t h, int route) {
    if (!h) return set_error(HODLR_EINVAL, "null handle");
    if (route < -1 || route > 2) return set_error(HODLR_EINVAL, "route must be -1, 0, 1 or 2");
    h->use_persistent = route;
    return HODLR_OK;
}

hodlr_status hodlr_autotune(hodlr_t h, int nrhs, int x_prec, int compute_prec,
                            hodlr_tuning* out, void* stream) {
    if (!h || !out) return set_error(HODLR_EINVAL, "null pointer argument");
    if (nrhs < 1) return set_error(HODLR_EINVAL, "nrhs must be >= 1");
    if (x_prec != HODLR_FP64 && x_prec != HODLR_FP32)
        return set_error(HODLR_EINVAL, "x_prec must be FP64 or FP32");
    if (compute_prec != HODLR_FP64 && compute_prec != HODLR_FP32)
        return set_error(HODLR_EINVAL, "compute_prec must be FP64 or FP32");
    if (h->opts.storage == HODLR_BF16 && compute_prec != HODLR_FP32)
        return set_error(HODLR_EINVAL, "BF16 factors are applied in FP32 arithmetic");
    if (h->opts.skeleton && compute_prec != HODLR_FP64)
        return set_error(HODLR_EINVAL, "the skeleton form is applied in FP64 arithmetic");
    for (int l = 1; l <= h->kappa; ++l)
        if (!h->lev[l].has_factors) return set_error(HODLR_EINVAL, "factors missing");
    return guarded([&] {
        hodlr::autotune(h, nrhs, x_prec, compute_prec, out, (hipStream_t)stream);
    });
}

hodlr_status hodlr_matvec_batch(int nslots, const hodlr_t* hs, const void* const* X,
                                const int64_t* ldx, const int* nrhs, int x_prec, void* const* Y,
                                const int64_t* ldy, void* stream) {
    if (nslots < 1 || !hs || !X || !ldx || !nrhs || !Y || !ldy)
        return set_error(HODLR_EINVAL, "null pointer argument or nslots < 1");
    if (x_prec != HODLR_FP64 && x_prec != HODLR_FP32)
        return set_error(HODLR_EINVAL, "x_prec must be FP64 or FP32");
    for (int t = 0; t < nslots; ++t) {
        hodlr_t h = hs[t];
        if (!h || !X[t] || !Y[t]) return set_error(HODLR_EINVAL, "null handle or vector");
        if (nrhs[t] < 1) return set_error(HODLR_EINVAL, "nrhs must be >= 1");
        if (ldx[t] < h->N || ldy[t] < h->N) return set_error(HODLR_EINVAL, "leading dimension < N");
        if (h->opts.storage != hs[0]->opts.storage || h->opts.storage == HODLR_BF16 ||
            h->opts.skeleton)
            return set_error(HODLR_EINVAL,
                             "a batch takes handles with FP64 or FP32 factors of one precision, "
                             "not the skeleton form");
        for (int u = 0; u < t; ++u)
            if (hs[u] == h) return set_error(HODLR_EINVAL, "a handle appears twice in the batch");
        for (int l = 1; l <= h->kappa; ++l)
            if (!h->lev[l].has_factors) return set_error(HODLR_EINVAL, "factors missing");
        if (!h->near_items) return set_error(HODLR_EINVAL, "factors missing");
    }
    return guarded([&] {
        hodlr::matvec_batch(nslots, hs, X, ldx, nrhs, x_prec, Y, ldy, nullptr,
                            (hipStream_t)stream);
    });
}

hodlr_status hodlr_matvec_noalloc(hodlr_t h, const void* X, int64_t ldx, int nrhs, int x_prec,
                                  void* Y, int64_t ldy, int compute_prec, void* stream) {
    return matvec_checked(h, X, ldx, nrhs, x_prec, Y, ldy, compute_prec, stream, nullptr, 0,
                          true);
}

hodlr_status hodlr_matvec_events(hodlr_t h, const void* X, int64_t ldx, int nrhs, int x_prec,
                                 void* Y, int64_t ldy, int compute_prec, void* stream,
                                 void* const* events, int nevents) {
    if (!events) return set_error(HODLR_EINVAL, "null events");
    return matvec_checked(h, X, ldx, nrhs, x_prec, Y, ldy, compute_prec, stream, events, nevents);
}

void hodlr_default_solve_opts(hodlr_solve_opts* o) {
    if (!o) return;
    o->tol = 1e-10;
    o->inner_tol = 1e-4;
    o->restart = 50;
    o->max_outer = 30;
    o->lo_compute = HODLR_FP32;
    o->use_initial_guess = 0;
}

hodlr_status hodlr_solve(hodlr_t hi, hodlr_t lo, double alpha, double beta, const double* F,
                         int64_t ldf, int nrhs, double* U, int64_t ldu,
                         const hodlr_solve_opts* opts, hodlr_solve_info* info, void* stream) {
    if (!hi || !lo || !F || !U) return set_error(HODLR_EINVAL, "null pointer argument");
    if (hi->N != lo->N || hi->d != lo->d)
        return set_error(HODLR_EINVAL, "hi and lo must be built on the same points");
    if (hi->opts.storage == HODLR_BF16)
        return set_error(HODLR_EINVAL, "hi must hold FP64 or FP32 factors (FP64 residuals)");
    if (nrhs < 1) return set_error(HODLR_EINVAL, "nrhs must be >= 1");
    if (ldf < hi->N || ldu < hi->N) return set_error(HODLR_EINVAL, "leading dimension < N");
    if (!std::isfinite(alpha) || !std::isfinite(beta))
        return set_error(HODLR_EINVAL, "alpha and beta must be finite");
    hodlr_solve_opts o;
    hodlr_default_solve_opts(&o);
    if (opts) o = *opts;
    if (!(o.tol > 0.0) || !(o.inner_tol > 0.0 && o.inner_tol < 1.0))
        return set_error(HODLR_EINVAL, "need tol > 0 and 0 < inner_tol < 1");
    if (o.restart < 1 || o.restart > 512) return set_error(HODLR_EINVAL, "restart must be 1..512");
    if (o.max_outer < 0) return set_error(HODLR_EINVAL, "max_outer must be >= 0");
    if (o.lo_compute != HODLR_FP64 && o.lo_compute != HODLR_FP32)
        return set_error(HODLR_EINVAL, "lo_compute must be FP64 or FP32");
    for (hodlr_t h : {hi, lo}) {
        for (int l = 1; l <= h->kappa; ++l)
            if (!h->lev[l].has_factors) return set_error(HODLR_EINVAL, "factors missing");
        if (!h->near_items) return set_error(HODLR_EINVAL, "factors missing");
    }
    hodlr_solve_info tmp{};
    return guarded([&] {
        hodlr::solve(hi, lo, alpha, beta, F, ldf, nrhs, U, ldu, o, info ? info : &tmp,
                     (hipStream_t)stream);
    });
}

void hodlr_server_default_opts(hodlr_server_opts* o) {
    if (!o) return;
    o->mem_budget_bytes = 0;
    o->max_concurrent = 8;
    o->max_batch_cols = 64;
    o->max_points = (int64_t)1 << 18;
    o->multiset = 0;
}

hodlr_status hodlr_server_create(const hodlr_server_opts* opts, hodlr_server_t* out) {
    if (!out) return set_error(HODLR_EINVAL, "null pointer argument");
    hodlr_server_opts o;
    hodlr_server_default_opts(&o);
    if (opts) o = *opts;
    if (o.max_concurrent < 1 || o.max_concurrent > 64)
        return set_error(HODLR_EINVAL, "max_concurrent must be 1..64");
    if (o.max_batch_cols < 1 || o.max_batch_cols > 1024)
        return set_error(HODLR_EINVAL, "max_batch_cols must be 1..1024");
    if (o.max_points < 1) return set_error(HODLR_EINVAL, "max_points must be >= 1");
    if (o.multiset != 0 && o.multiset != 1) return set_error(HODLR_EINVAL, "multiset must be 0 or 1");
    return guarded([&] {
        if (o.mem_budget_bytes == 0) {
            size_t fr = 0, tot = 0;
            HIP_CHECK(hipMemGetInfo(&fr, &tot));
            o.mem_budget_bytes = fr / 10 * 9;
        }
        const hodlr_status st = hodlr::server_create(o, out);
        if (st != HODLR_OK) hodlr::fail(st, "server creation failed");
    });
}

hodlr_status hodlr_server_add_set(hodlr_server_t srv, const double* points, int64_t N, int d,
                                  const hodlr_kernel* kernel, int leaf_size, double tol,
                                  const hodlr_opts* opts, int* set_id) {
    if (!srv || !set_id) return set_error(HODLR_EINVAL, "null pointer argument");
    hodlr_opts o;
    hodlr_default_opts(&o);
    if (opts) o = *opts;
    o.mem_budget_bytes = hodlr::server_room(srv);
    if (o.mem_budget_bytes == 0) return set_error(HODLR_ENOMEM, "server memory budget exhausted");
    hodlr_t h = nullptr;
    const hodlr_status st = hodlr_build(points, N, d, kernel, leaf_size, tol, &o, nullptr, &h);
    if (st != HODLR_OK) return st;
    return guarded([&] {
        try {
            // size the product workspace once for every batch width it will see
            const int cols = hodlr::server_batch_cols(srv);
            for (int prec : {HODLR_FP64, HODLR_FP32}) {
                if (h->opts.storage == HODLR_BF16 && prec == HODLR_FP64) continue;
                hodlr::reserve_workspace(h, 1, prec, nullptr);
                hodlr::reserve_workspace(h, cols, prec, nullptr);
            }
        } catch (...) {
            hodlr_destroy(h);
            throw;
        }
        *set_id = hodlr::server_add(srv, h);
    });
}

hodlr_status hodlr_server_submit(hodlr_server_t srv, const hodlr_request* req, int64_t* id) {
    if (!srv || !req || !id || !req->X || !req->Y)
        return set_error(HODLR_EINVAL, "null pointer argument");
    if (req->kind != HODLR_REQ_MATVEC && req->kind != HODLR_REQ_SOLVE)
        return set_error(HODLR_EINVAL, "unknown request kind");
    if (req->nrhs < 1) return set_error(HODLR_EINVAL, "nrhs must be >= 1");
    if (req->kind == HODLR_REQ_SOLVE &&
        (!(req->tol > 0) || !std::isfinite(req->alpha) || !std::isfinite(req->beta)))
        return set_error(HODLR_EINVAL, "solve needs tol > 0 and finite alpha, beta");
    std::string err;
    const hodlr_status st = hodlr::server_submit(srv, *req, id, err);
    if (st != HODLR_OK) return set_error(st, err);
    g_last_error.clear();
    return HODLR_OK;
}

hodlr_status hodlr_server_wait(hodlr_server_t srv, int64_t id, double* queue_us, double* run_us) {
    if (!srv) return set_error(HODLR_EINVAL, "null server");
    std::string err;
    const hodlr_status st = hodlr::server_wait(srv, id, 1, nullptr, queue_us, run_us, err);
    if (st != HODLR_OK) return set_error(st, err);
    g_last_error.clear();
    return HODLR_OK;
}

hodlr_status hodlr_server_poll(hodlr_server_t srv, int64_t id, int* done, double* queue_us,
                               double* run_us) {
    if (!srv || !done) return set_error(HODLR_EINVAL, "null pointer argument");
    std::string err;
    const hodlr_status st = hodlr::server_wait(srv, id, 0, done, queue_us, run_us, err);
    if (st != HODLR_OK) return set_error(st, err);
    g_last_error.clear();
    return HODLR_OK;
}

hodlr_status hodlr_server_get_stats(hodlr_server_t srv, hodlr_server_stats* stats) {
    if (!srv || !stats) return set_error(HODLR_EINVAL, "null pointer argument");
    hodlr::server_stats(srv, stats);
    return HODLR_OK;
}

void hodlr_server_destroy(hodlr_server_t srv) {
    if (srv) hodlr::server_destroy(srv);
}

hodlr_status hodlr_get_info(hodlr_t h, hodlr_info* info) {
    if (!h || !info) return set_error(HODLR_EINVAL, "null pointer argument");
    std::memset(info, 0, sizeof(*info));
    info->N = h->N;
    info->d = h->d;
    info->kappa = h->kappa;
    info->lmax = h->lmax;
    info->symmetric = h->opts.symmetric;
    info->storage = h->opts.storage;
    for (int a = 0; a < h->d; ++a) info->domain_lo[a] = h->lo[a];
    info->domain_side = h->side;
    for (int l = 0; l <= h->kappa; ++l) {
        info->nboxes[l] = h->lev[l].nb;
        info->il_entries[l] = h->lev[l].nnz;
        info->stored_blocks[l] = h->lev[l].nblk;
        int32_t rmin = INT32_MAX, rmax = 0;
        double rs = 0;
        int64_t fe = 0;
        for (int64_t b = h->lev[l].blk0; b < h->lev[l].blk0 + h->lev[l].nblk; ++b) {
            const auto& bd = h->hblocks[b];
            rmin = std::min(rmin, bd.rank);
            rmax = std::max(rmax, bd.rank);
            rs += bd.rank;
            fe += (int64_t)std::max(bd.rank, 0) *
                  (h->opts.skeleton ? (int64_t)std::max(bd.rank, 0) : (int64_t)(bd.m + bd.n));
        }
        info->rank_min[l] = h->lev[l].nblk ? rmin : 0;
        info->rank_max[l] = rmax;
        info->rank_mean[l] = h->lev[l].nblk ? rs / h->lev[l].nblk : 0.0;
        info->factor_elems[l] = fe;
    }
    for (int c = 0; c < hodlr::kApplyClasses && c < 8; ++c) {
        info->class_blocks[c] = (int64_t)h->class_off.size() > c + 1
                                    ? h->class_off[c + 1] - h->class_off[c]
                                    : 0;
        info->class_factor_elems[c] = h->cls_felems[c];
        info->class_vector_elems[c] = h->cls_velems[c];
    }
    info->split_blocks = h->split_blocks;
    info->split_factor_elems = h->split_felems;
    if (h->opts.storage == HODLR_BF16) {
        for (int c = 0; c < 4; ++c) {
            info->mfma_proj_jobs[c] = h->mjob_count[c];
            info->mfma_proj_factor_elems[c] = h->mjob_felems[c];
            info->mfma_proj_vector_elems[c] = h->mjob_velems[c];
        }
        info->mfma_expand_factor_elems = h->mexp_felems;
        info->mfma_proj_elems = h->mt_total;
    }
    info->near_entries = 0;
    for (int l = 0; l <= h->kappa; ++l) info->near_entries += h->lev[l].near_nnz;
    info->near_pairs = h->near_pairs;
    info->device_bytes = h->device_bytes;
    for (int i = 0; i < 4; ++i) info->build_ms[i] = h->build_ms[i];
    return HODLR_OK;
}

hodlr_status hodlr_export_tree(hodlr_t h, int64_t* perm, uint64_t* keys) {
    if (!h) return set_error(HODLR_EINVAL, "null handle");
    return guarded([&] {
        if (perm) {
            std::vector<int32_t> p(h->N);
            HIP_CHECK(hipMemcpy(p.data(), h->perm, sizeof(int32_t) * h->N, hipMemcpyDeviceToHost));
            for (int64_t i = 0; i < h->N; ++i) perm[i] = p[i];
        }
        if (keys)
            HIP_CHECK(hipMemcpy(keys, h->keys, sizeof(uint64_t) * h->N, hipMemcpyDeviceToHost));
    });
}

hodlr_status hodlr_export_boxes(hodlr_t h, int level, int64_t* start, uint64_t* key,
                                int32_t* coord) {
    if (!h) return set_error(HODLR_EINVAL, "null handle");
    if (level < 0 || level > h->kappa) return set_error(HODLR_EINVAL, "level out of range");
    return guarded([&] {
        const auto& Lv = h->lev[level];
        if (start)
            for (int64_t b = 0; b <= Lv.nb; ++b) start[b] = Lv.hstart[b];
        if (key) HIP_CHECK(hipMemcpy(key, Lv.key, sizeof(uint64_t) * Lv.nb, hipMemcpyDeviceToHost));
        if (coord)
            HIP_CHECK(hipMemcpy(coord, Lv.coord, sizeof(int32_t) * Lv.nb * h->d,
                                hipMemcpyDeviceToHost));
    });
}

hodlr_status hodlr_export_il(hodlr_t h, int level, int64_t* nnz, int64_t* ptr, int32_t* col) {
    if (!h) return set_error(HODLR_EINVAL, "null handle");
    if (level < 1 || level > h->kappa) return set_error(HODLR_EINVAL, "level out of range");
    return guarded([&] {
        const auto& Lv = h->lev[level];
        if (nnz) *nnz = Lv.nnz;
        if (ptr)
            HIP_CHECK(hipMemcpy(ptr, Lv.il_ptr, sizeof(int64_t) * (Lv.nb + 1), hipMemcpyDeviceToHost));
        if (col && Lv.nnz)
            HIP_CHECK(hipMemcpy(col, Lv.il_col, sizeof(int32_t) * Lv.nnz, hipMemcpyDeviceToHost));
    });
}

hodlr_status hodlr_export_near(hodlr_t h, int64_t* nnz, int64_t* ptr, int32_t* col) {
    if (!h) return set_error(HODLR_EINVAL, "null handle");
    return guarded([&] {
        const auto& Lv = h->lev[h->kappa];
        if (nnz) *nnz = h->near_nnz;
        if (ptr)
            HIP_CHECK(hipMemcpy(ptr, h->near_ptr, sizeof(int64_t) * (Lv.nb + 1),
                                hipMemcpyDeviceToHost));
        if (col && h->near_nnz)
            HIP_CHECK(hipMemcpy(col, h->near_col, sizeof(int32_t) * h->near_nnz,
                                hipMemcpyDeviceToHost));
    });
}

hodlr_status hodlr_export_near_level(hodlr_t h, int level, int64_t* nnz, int64_t* ptr,
                                     int32_t* col) {
    if (!h) return set_error(HODLR_EINVAL, "null handle");
    if (level < 0 || level > h->kappa) return set_error(HODLR_EINVAL, "level out of range");
    return guarded([&] {
        const auto& Lv = h->lev[level];
        if (nnz) *nnz = Lv.near_nnz;
        if (ptr)
            HIP_CHECK(hipMemcpy(ptr, Lv.near_ptr, sizeof(int64_t) * (Lv.nb + 1),
                                hipMemcpyDeviceToHost));
        if (col && Lv.near_nnz)
            HIP_CHECK(hipMemcpy(col, Lv.near_col, sizeof(int32_t) * Lv.near_nnz,
                                hipMemcpyDeviceToHost));
    });
}

hodlr_status hodlr_export_box_flags(hodlr_t h, int level, uint8_t* flags) {
    if (!h) return set_error(HODLR_EINVAL, "null handle");
    if (level < 0 || level > h->kappa) return set_error(HODLR_EINVAL, "level out of range");
    return guarded([&] {
        const auto& Lv = h->lev[level];
        if (flags && Lv.nb) std::copy(Lv.hflags.begin(), Lv.hflags.end(), flags);
    });
}

hodlr_status hodlr_export_factors(hodlr_t h, int level, int32_t* ranks, int64_t* u_elems,
                                  int64_t* v_elems, double* U, double* V) {
    if (!h) return set_error(HODLR_EINVAL, "null handle");
    if (level < 1 || level > h->kappa) return set_error(HODLR_EINVAL, "level out of range");
    if (h->opts.skeleton && (U || V))
        return set_error(HODLR_EUNSUPPORTED, "skeleton form: only the ranks can be exported");
    return guarded([&] { hodlr::export_level(h, level, ranks, u_elems, v_elems, U, V, nullptr); });
}

hodlr_status hodlr_import_factors(hodlr_t h, int level, const int32_t* ranks, const double* U,
                                  const double* V) {
    if (!h || !ranks) return set_error(HODLR_EINVAL, "null pointer argument");
    if (level < 1 || level > h->kappa) return set_error(HODLR_EINVAL, "level out of range");
    if (h->opts.skeleton) return set_error(HODLR_EUNSUPPORTED, "skeleton form: no factor import");
    return guarded([&] { hodlr::import_level(h, level, ranks, U, V, nullptr); });
}

void hodlr_destroy(hodlr_t h) {
    if (!h) return;
    (void)hipDeviceSynchronize();
    free_all(h);
    delete h;
}

const char* hodlr_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"
