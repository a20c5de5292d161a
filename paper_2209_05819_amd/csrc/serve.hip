// Serving engine: resident HODLRdD representations of several point sets and
// a request loop with continuous batching.
//
//   - A set's tree, lists and factors stay on the device from
//     hodlr_server_add_set until the server is destroyed; the device memory of
//     all sets plus the running requests' workspaces is kept under a budget.
//   - Requests (products and solves) queue in arrival order.  A scheduler
//     thread starts work whenever a set is idle and one of max_concurrent
//     stream slots is free: all queued products of that set (in order, up to
//     max_batch_cols columns) are gathered into one product, and the queued
//     products of other idle sets with the same factor precision (FP64 or
//     FP32) join the same launch (one persistent launch applies every set of
//     the batch, up to kBatchSets sets and the slot's buffer); a solve runs
//     on a worker thread on its own slot.  Work on different slots overlaps
//     on the device; requests arriving while others run are admitted as
//     slots and memory free up.
//   - Completion is observed through an event per slot; each request records
//     its queueing and running time.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <vector>

#include "hodlr_impl.hpp"

namespace {

using clk = std::chrono::steady_clock;

double us_between(clk::time_point a, clk::time_point b) {
    return std::chrono::duration<double, std::micro>(b - a).count();
}

struct Req {
    int64_t id = 0;
    hodlr_request r{};
    hipEvent_t ready = nullptr;   // recorded on the request's stream at submission
    int state = 0;   // 0 queued, 1 running, 2 done
    hodlr_status st = HODLR_OK;
    std::string msg;
    clk::time_point t_submit, t_start, t_done;
};

struct Set {
    hodlr_t h = nullptr;
    bool busy = false;
};

constexpr int kBatchSets = 16;        // sets one batched launch applies at most
constexpr size_t kBatchSegs = 8192;   // claim-queue segments of one batched launch

struct Slot {
    hipStream_t s = nullptr;
    hipEvent_t ev = nullptr;
    double* xb = nullptr;   // batch input, max_points x max_batch_cols elements
    double* yb = nullptr;
    void* bt = nullptr;     // device tables of batched launches
    bool busy = false;
    // the running job: its sets and, per set, its requests (in order)
    std::vector<int> sets;
    bool solve = false;
    std::vector<Req*> reqs;
    std::vector<int> req_set;      // position in `sets` of each request
    std::vector<int64_t> xoff;     // element offset of each request's columns in xb / yb
    size_t bytes = 0;
    std::thread worker;
    std::atomic<bool> worker_done{false};
};

}  // namespace

struct hodlr_server_s {
    hodlr_server_opts o{};
    std::mutex mu;
    std::condition_variable cv;   // request state changes
    std::vector<Set> sets;
    std::deque<Req*> queue;
    std::map<int64_t, std::unique_ptr<Req>> reqs;
    std::vector<std::unique_ptr<Slot>> slots;
    std::thread sched;
    bool stop = false;
    int64_t next_id = 1;
    size_t used = 0;   // resident sets + running workspaces
    hodlr_server_stats stats{};
    int running = 0;
};

namespace hodlr {

namespace {

void finish_job(hodlr_server_s* S, Slot& sl, hodlr_status st, const std::string& msg) {
    const auto now = clk::now();
    for (size_t k = 0; k < sl.reqs.size(); ++k) {
        Req* q = sl.reqs[k];
        q->t_done = now;
        q->state = 2;
        q->st = st;
        q->msg = msg;
        if (st == HODLR_OK)
            ++S->stats.completed;
        else
            ++S->stats.failed;
    }
    for (int st : sl.sets) S->sets[st].busy = false;
    S->used -= sl.bytes;
    sl.bytes = 0;
    sl.busy = false;
    sl.reqs.clear();
    sl.req_set.clear();
    sl.xoff.clear();
    sl.sets.clear();
    --S->running;
}

// start the products of slot sl (called with the lock held): the requests
// of each set side by side in the slot's buffer (set g's columns at offset
// xoff), one product per set, or one batched launch for several sets
void launch_products(hodlr_server_s* S, Slot& sl) {
    const int ng = (int)sl.sets.size();
    std::vector<hodlr_t> hs(ng);
    std::vector<int> cols(ng, 0);
    std::vector<int64_t> goff(ng, 0);
    for (int g = 0; g < ng; ++g) hs[g] = S->sets[sl.sets[g]].h;
    // element offsets: sets one after the other, each set's requests in order
    int64_t off = 0;
    for (int g = 0; g < ng; ++g) {
        goff[g] = off;
        for (size_t k = 0; k < sl.reqs.size(); ++k)
            if (sl.req_set[k] == g) {
                sl.xoff[k] = off;
                off += hs[g]->N * sl.reqs[k]->r.nrhs;
                cols[g] += sl.reqs[k]->r.nrhs;
            }
    }
    try {
        // X is read only after the work queued before submission on its stream
        for (Req* q : sl.reqs) HIP_CHECK(hipStreamWaitEvent(sl.s, q->ready, 0));
        for (size_t k = 0; k < sl.reqs.size(); ++k) {
            const int64_t N = hs[sl.req_set[k]]->N;
            HIP_CHECK(hipMemcpyAsync(sl.xb + sl.xoff[k], sl.reqs[k]->r.X,
                                     sizeof(double) * N * sl.reqs[k]->r.nrhs,
                                     hipMemcpyDeviceToDevice, sl.s));
        }
        if (ng == 1) {
            hodlr_t h = hs[0];
            const int prec = h->opts.storage == HODLR_FP64 ? HODLR_FP64 : HODLR_FP32;
            matvec(h, sl.xb, h->N, cols[0], HODLR_FP64, sl.yb, h->N, prec, nullptr, 0, sl.s);
        } else {
            std::vector<const void*> X(ng);
            std::vector<void*> Y(ng);
            std::vector<int64_t> ld(ng);
            for (int g = 0; g < ng; ++g) {
                X[g] = sl.xb + goff[g];
                Y[g] = sl.yb + goff[g];
                ld[g] = hs[g]->N;
            }
            matvec_batch_async(ng, hs.data(), X.data(), ld.data(), cols.data(), HODLR_FP64,
                               Y.data(), ld.data(), sl.bt, sl.s);
        }
        for (size_t k = 0; k < sl.reqs.size(); ++k) {
            const int64_t N = hs[sl.req_set[k]]->N;
            HIP_CHECK(hipMemcpyAsync(sl.reqs[k]->r.Y, sl.yb + sl.xoff[k],
                                     sizeof(double) * N * sl.reqs[k]->r.nrhs,
                                     hipMemcpyDeviceToDevice, sl.s));
        }
        HIP_CHECK(hipEventRecord(sl.ev, sl.s));
    } catch (const Error& e) {
        (void)hipStreamSynchronize(sl.s);
        finish_job(S, sl, e.code, e.msg);
        return;
    }
    ++S->stats.launches;
    if (sl.reqs.size() > 1) S->stats.batched_requests += (int64_t)sl.reqs.size();
    if (ng > 1) ++S->stats.multiset_launches;
}

void launch_solve(hodlr_server_s* S, Slot& sl) {
    hodlr_t h = S->sets[sl.sets[0]].h;
    Req* q = sl.reqs[0];
    sl.worker_done = false;
    ++S->stats.launches;
    sl.worker = std::thread([S, &sl, h, q] {
        hodlr_status st = HODLR_OK;
        std::string msg;
        try {
            hodlr_solve_opts so;
            hodlr_default_solve_opts(&so);
            so.tol = q->r.tol;
            so.inner_tol = 1e-3;
            so.restart = 30;
            so.max_outer = 40;
            so.lo_compute = HODLR_FP32;
            hodlr_solve_info info{};
            HIP_CHECK(hipStreamWaitEvent(sl.s, q->ready, 0));
            solve(h, h, q->r.alpha, q->r.beta, q->r.X, h->N, q->r.nrhs, q->r.Y, h->N, so, &info,
                  sl.s);
            if (!info.converged) {
                st = HODLR_EUNSUPPORTED;
                msg = "solve did not reach the tolerance";
            }
        } catch (const Error& e) {
            st = e.code;
            msg = e.msg;
        } catch (...) {
            st = HODLR_EDEVICE;
            msg = "unexpected solver error";
        }
        std::lock_guard<std::mutex> lk(S->mu);
        q->st = st;
        q->msg = msg;
        sl.worker_done = true;
        S->cv.notify_all();
    });
}

void scheduler(hodlr_server_s* S) {
    std::unique_lock<std::mutex> lk(S->mu);
    for (;;) {
        bool progress = false;
        // completions
        for (auto& up : S->slots) {
            Slot& sl = *up;
            if (!sl.busy) continue;
            if (sl.solve) {
                if (sl.worker_done) {
                    lk.unlock();
                    sl.worker.join();
                    lk.lock();
                    const hodlr_status st = sl.reqs[0]->st;
                    const std::string msg = sl.reqs[0]->msg;
                    finish_job(S, sl, st, msg);
                    progress = true;
                }
            } else {
                const hipError_t e = hipEventQuery(sl.ev);
                if (e == hipSuccess) {
                    finish_job(S, sl, HODLR_OK, "");
                    progress = true;
                } else if (e != hipErrorNotReady) {
                    finish_job(S, sl, HODLR_EDEVICE, hipGetErrorString(e));
                    progress = true;
                }
            }
        }
        if (progress) S->cv.notify_all();
        if (S->stop && S->queue.empty() && S->running == 0) break;
        // dispatch in arrival order
        for (size_t qi = 0; qi < S->queue.size();) {
            Req* q = S->queue[qi];
            Set& st = S->sets[q->r.set];
            Slot* free_slot = nullptr;
            for (auto& up : S->slots)
                if (!up->busy) {
                    free_slot = up.get();
                    break;
                }
            if (!free_slot) break;
            if (st.busy) {
                ++qi;
                continue;
            }
            Slot& sl = *free_slot;
            sl.reqs.clear();
            sl.req_set.clear();
            sl.sets.clear();
            size_t bytes = 0;
            if (q->r.kind == HODLR_REQ_SOLVE) {
                bytes = sizeof(double) * (size_t)st.h->N * q->r.nrhs * (30 + 5);
                if (S->used + bytes > S->o.mem_budget_bytes && S->running > 0) {
                    ++qi;
                    continue;
                }
                sl.sets.push_back(q->r.set);
                sl.reqs.push_back(q);
                sl.req_set.push_back(0);
                S->queue.erase(S->queue.begin() + qi);
            } else {
                // this set's queued products, in order, up to the column cap;
                // then those of other idle sets with the same factor precision
                const size_t cap = (size_t)S->o.max_points * S->o.max_batch_cols;
                size_t elems = 0;
                const int prec = st.h->opts.storage;
                const bool batchable = S->o.multiset && (prec == HODLR_FP64 || prec == HODLR_FP32) &&
                                       !st.h->opts.skeleton;
                auto take_set = [&](int set) {
                    const int64_t N = S->sets[set].h->N;
                    int cols = 0;
                    std::vector<size_t> picked;
                    for (size_t k = 0; k < S->queue.size(); ++k) {
                        Req* p = S->queue[k];
                        if (p->r.set == set && p->r.kind == HODLR_REQ_MATVEC &&
                            cols + p->r.nrhs <= S->o.max_batch_cols &&
                            elems + (size_t)N * (cols + p->r.nrhs) <= cap) {
                            cols += p->r.nrhs;
                            picked.push_back(k);
                        }
                    }
                    if (picked.empty()) return;
                    const int g = (int)sl.sets.size();
                    sl.sets.push_back(set);
                    for (size_t k : picked) {
                        sl.reqs.push_back(S->queue[k]);
                        sl.req_set.push_back(g);
                    }
                    for (size_t t = picked.size(); t-- > 0;)
                        S->queue.erase(S->queue.begin() + picked[t]);
                    elems += (size_t)N * cols;
                };
                take_set(q->r.set);
                if (batchable) {
                    for (size_t k = 0; k < S->queue.size() && (int)sl.sets.size() < kBatchSets;) {
                        Req* p = S->queue[k];
                        const Set& ps = S->sets[p->r.set];
                        bool mine = false;
                        for (int x : sl.sets) mine = mine || x == p->r.set;
                        if (p->r.kind == HODLR_REQ_MATVEC && !mine && !ps.busy &&
                            ps.h->opts.storage == prec && !ps.h->opts.skeleton &&
                            elems + (size_t)ps.h->N * p->r.nrhs <= cap) {
                            const size_t before = S->queue.size();
                            take_set(p->r.set);
                            if (S->queue.size() == before) ++k;   // nothing fitted
                            // requests before k stay; k now names the next one
                        } else {
                            ++k;
                        }
                    }
                }
                sl.xoff.assign(sl.reqs.size(), 0);
            }
            const auto now = clk::now();
            for (Req* p : sl.reqs) {
                p->state = 1;
                p->t_start = now;
            }
            for (int x : sl.sets) S->sets[x].busy = true;
            sl.busy = true;
            sl.solve = q->r.kind == HODLR_REQ_SOLVE;
            sl.bytes = bytes;
            S->used += bytes;
            ++S->running;
            S->stats.max_concurrent = std::max<int64_t>(S->stats.max_concurrent, S->running);
            if (sl.solve)
                launch_solve(S, sl);
            else
                launch_products(S, sl);
            progress = true;
            // qi now points at the next unhandled request
        }
        if (!progress) {
            if (S->running == 0 && S->queue.empty() && !S->stop)
                S->cv.wait(lk);
            else
                S->cv.wait_for(lk, std::chrono::microseconds(20));
        }
    }
}

}  // namespace

}  // namespace hodlr

namespace hodlr {
// used by api.hip
hodlr_status server_create(const hodlr_server_opts& o, hodlr_server_t* out) {
    auto S = std::make_unique<hodlr_server_s>();
    S->o = o;
    for (int i = 0; i < o.max_concurrent; ++i) {
        auto sl = std::make_unique<Slot>();
        HIP_CHECK(hipStreamCreateWithFlags(&sl->s, hipStreamNonBlocking));
        HIP_CHECK(hipEventCreateWithFlags(&sl->ev, hipEventDisableTiming));
        const size_t n = (size_t)o.max_points * o.max_batch_cols;
        if (hipMalloc(&sl->xb, sizeof(double) * std::max<size_t>(n, 1)) != hipSuccess ||
            hipMalloc(&sl->yb, sizeof(double) * std::max<size_t>(n, 1)) != hipSuccess) {
            (void)hipGetLastError();
            for (auto& s2 : S->slots) {
                (void)hipFree(s2->xb);
                (void)hipFree(s2->yb);
            }
            (void)hipFree(sl->xb);
            fail(HODLR_ENOMEM, "server batch buffers");
        }
        S->used += 2 * sizeof(double) * n;
        sl->bt = batch_tables_create(kBatchSets, kBatchSegs);
        S->slots.push_back(std::move(sl));
    }
    if (S->used > o.mem_budget_bytes) fail(HODLR_ENOMEM, "budget below the batch buffers");
    hodlr_server_s* raw = S.release();
    raw->sched = std::thread(scheduler, raw);
    *out = raw;
    return HODLR_OK;
}

void server_destroy(hodlr_server_t S) {
    {
        std::lock_guard<std::mutex> lk(S->mu);
        S->stop = true;
    }
    S->cv.notify_all();
    S->sched.join();
    for (auto& sl : S->slots) {
        (void)hipStreamSynchronize(sl->s);
        (void)hipFree(sl->xb);
        (void)hipFree(sl->yb);
        batch_tables_destroy(sl->bt);
        (void)hipEventDestroy(sl->ev);
        (void)hipStreamDestroy(sl->s);
    }
    for (auto& st : S->sets) hodlr_destroy(st.h);
    for (auto& kv : S->reqs) (void)hipEventDestroy(kv.second->ready);
    delete S;
}

// registers a built handle (the caller built it under the remaining budget)
int server_add(hodlr_server_t S, hodlr_t h) {
    std::lock_guard<std::mutex> lk(S->mu);
    S->sets.push_back(Set{h, false});
    S->used += h->device_bytes;
    return (int)S->sets.size() - 1;
}

size_t server_room(hodlr_server_t S) {
    std::lock_guard<std::mutex> lk(S->mu);
    return S->o.mem_budget_bytes > S->used ? S->o.mem_budget_bytes - S->used : 0;
}

int server_batch_cols(hodlr_server_t S) { return S->o.max_batch_cols; }

hodlr_status server_submit(hodlr_server_t S, const hodlr_request& r, int64_t* id, std::string& err) {
    std::lock_guard<std::mutex> lk(S->mu);
    if (r.set < 0 || r.set >= (int)S->sets.size()) {
        err = "unknown set";
        return HODLR_EINVAL;
    }
    hodlr_t h = S->sets[r.set].h;
    if (r.nrhs > S->o.max_batch_cols) {
        err = "nrhs exceeds max_batch_cols";
        return HODLR_EINVAL;
    }
    if (h->N > S->o.max_points) {
        err = "set larger than max_points";
        return HODLR_EINVAL;
    }
    if (r.kind == HODLR_REQ_SOLVE && h->opts.storage == HODLR_BF16) {
        err = "solves need FP64 or FP32 factors";
        return HODLR_EINVAL;
    }
    auto q = std::make_unique<Req>();
    if (hipEventCreateWithFlags(&q->ready, hipEventDisableTiming) != hipSuccess ||
        hipEventRecord(q->ready, (hipStream_t)r.stream) != hipSuccess) {
        (void)hipGetLastError();
        if (q->ready) (void)hipEventDestroy(q->ready);
        err = "could not record the request's stream";
        return HODLR_EDEVICE;
    }
    q->id = S->next_id++;
    q->r = r;
    q->t_submit = clk::now();
    S->queue.push_back(q.get());
    *id = q->id;
    S->reqs[q->id] = std::move(q);
    ++S->stats.submitted;
    S->cv.notify_all();
    return HODLR_OK;
}

hodlr_status server_wait(hodlr_server_t S, int64_t id, int block, int* done, double* queue_us,
                         double* run_us, std::string& err) {
    std::unique_lock<std::mutex> lk(S->mu);
    auto it = S->reqs.find(id);
    if (it == S->reqs.end()) {
        err = "unknown request";
        return HODLR_EINVAL;
    }
    Req* q = it->second.get();
    if (block) S->cv.wait(lk, [&] { return q->state == 2; });
    if (done) *done = q->state == 2;
    if (q->state != 2) return HODLR_OK;
    if (queue_us) *queue_us = us_between(q->t_submit, q->t_start);
    if (run_us) *run_us = us_between(q->t_start, q->t_done);
    const hodlr_status st = q->st;
    err = q->msg;
    (void)hipEventDestroy(q->ready);
    S->reqs.erase(it);   // a finished request is reported once
    return st;
}

void server_stats(hodlr_server_t S, hodlr_server_stats* st) {
    std::lock_guard<std::mutex> lk(S->mu);
    *st = S->stats;
    st->used_bytes = S->used;
    st->budget_bytes = S->o.mem_budget_bytes;
    st->sets = (int)S->sets.size();
}

}  // namespace hodlr
