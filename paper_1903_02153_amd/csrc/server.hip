// Serving loop: several resident (tree, operators) models, requests of
// different N and r, continuous batching along the right-hand-side axis
// (the multiple-RHS grouping of Section 2.5 applied across requests).
//
// A scheduler thread repeatedly
//   1. retires finished batches (event query) and wakes their waiters;
//   2. takes the oldest pending request, gathers every pending request of
//      the same model in arrival order while the total r fits r_max, and
//      rounds the total up to a power of two (the batch width R);
//   3. admits the batch when a slot (own stream, own plan and staging
//      buffers) is free and the slots' device memory stays within the HBM
//      budget, else waits for a retirement;
//   4. packs the requests' sigma columns into the slot's N x R staging
//      matrix (padding columns zero), runs the plan, unpacks phi columns.
// Batches on different slots run concurrently on separate streams.  Plans
// (workspace, staging and the captured graph of one (model, R)) live in a
// cache shared by the slots, reused while idle and evicted least recently
// used first when the budget needs room.
//
// Batch invariance: every plan the server makes splits the M2L slot range
// over the same kServeSplit workgroups and, from R = 2 on, runs the near
// field on MFMA (a batch of width 1 -- one request with r = 1 -- takes the
// per-lane near field, the faster one for a single column).  With those
// fixed, the arithmetic of one right-hand side does not depend on the batch
// width R >= 2 or on the other columns (P2M/M2M/L2L work per (cell,
// column), the (de)compression GEMMs, the M2L and the MFMA near field
// accumulate each column in a fixed order), so a request's phi is
// bit-identical to a lone plan execution with m2l_split = kServeSplit and
// p2p_mfma = 2 whatever batch of width >= 2 it ran in, and to one with
// p2p_mfma = 1 when it ran alone at R = 1.
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <unordered_map>

#include "common.h"

namespace bbfmm {
namespace {

constexpr int kThreads = 256;
constexpr int kServeSplit = 2;

// dst[i][c0 + c] = src[i][c] for c < rs; dst has R columns
__global__ void __launch_bounds__(kThreads)
k_pack(const float *src, int64_t n, int rs, float *dst, int R, int c0) {
    const int64_t g = int64_t(blockIdx.x) * kThreads + threadIdx.x;
    if (g >= n * rs) return;
    const int64_t i = g / rs;
    const int c = int(g % rs);
    dst[i * R + c0 + c] = src[g];
}

// dst[i][c] = 0 for c0 <= c < R
__global__ void __launch_bounds__(kThreads)
k_zero_cols(int64_t n, float *dst, int R, int c0) {
    const int w = R - c0;
    const int64_t g = int64_t(blockIdx.x) * kThreads + threadIdx.x;
    if (g >= n * w) return;
    dst[(g / w) * R + c0 + g % w] = 0.f;
}

// dst[i][c] = src[i][c0 + c]
__global__ void __launch_bounds__(kThreads)
k_unpack(const float *src, int64_t n, int R, int c0, float *dst, int rs) {
    const int64_t g = int64_t(blockIdx.x) * kThreads + threadIdx.x;
    if (g >= n * rs) return;
    const int64_t i = g / rs;
    const int c = int(g % rs);
    dst[g] = src[i * R + c0 + c];
}

inline int grid(int64_t n) { return int(ceil_div(n, kThreads)); }

double now_s() {
    using namespace std::chrono;
    return duration<double>(steady_clock::now().time_since_epoch()).count();
}

struct Request {
    uint64_t id = 0;
    int model = 0;
    const float *sigma = nullptr;
    float *phi = nullptr;
    int64_t r = 0;
    double t_submit = 0, t_admit = 0, t_done = 0;
    int32_t batch_r = 0, slot = -1;
    bool done = false;
    bbfmm_status status = BBFMM_OK;
    std::string error;
};

struct Model {
    const bbfmm_tree *tree;
    const bbfmm_ops *ops;
};

// A plan and its N x R staging matrices for one (model, R); used by one
// slot at a time, cached while idle.
struct Entry {
    int model = -1, R = 0;
    Plan *plan = nullptr;
    DBuf<float> sig, phi;
    int64_t bytes = 0;                 // plan workspace + staging
    uint64_t last_use = 0;
    bool busy = false;
    ~Entry() { plan_destroy(plan); }
};

struct Slot {
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    bool busy = false;
    Entry *entry = nullptr;
    std::vector<Request *> batch;
};

}  // namespace

struct Server {
    int64_t budget;
    int max_inflight, r_max;
    std::vector<Model> models;
    std::vector<Slot> slots;
    std::vector<std::unique_ptr<Entry>> cache;
    std::map<std::pair<int, int>, int64_t> need;   // bytes of a (model, R) entry, once known
    std::deque<Request *> pending;
    std::unordered_map<uint64_t, std::unique_ptr<Request>> requests;
    uint64_t next_id = 1, tick = 0;
    int64_t in_use = 0;
    bbfmm_server_stats st{};
    int device = 0;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::thread worker;
    bool stop = false;
    std::string fatal;

    int waiters = 0;                   // threads inside bbfmm_server_wait

    ~Server() {
        {
            std::lock_guard<std::mutex> lk(mu);
            stop = true;
        }
        cv_work.notify_all();
        if (worker.joinable()) worker.join();
        for (Slot &s : slots)
            if (s.stream) (void)hipStreamSynchronize(s.stream);
        {
            // finish the batches that ran, cancel what never started, and
            // let every thread blocked in wait return before anything it
            // waits on is destroyed
            std::unique_lock<std::mutex> lk(mu);
            retire();
            for (Request *rq : pending) {
                rq->status = BBFMM_ERR_CANCELLED;
                rq->error = "the server was destroyed before the request ran";
                rq->done = true;
            }
            pending.clear();
            cv_done.notify_all();
            cv_done.wait(lk, [&] { return waiters == 0; });
        }
        cache.clear();
        for (Slot &s : slots) {
            if (s.done) (void)hipEventDestroy(s.done);
            if (s.stream) (void)hipStreamDestroy(s.stream);
        }
    }

    // called with mu held
    void retire() {
        for (size_t k = 0; k < slots.size(); ++k) {
            Slot &s = slots[k];
            if (!s.busy) continue;
            const hipError_t q = hipEventQuery(s.done);
            if (q == hipErrorNotReady) continue;
            const double t = now_s();
            for (Request *rq : s.batch) {
                rq->t_done = t;
                rq->done = true;
                ++st.requests_done;
                if (q != hipSuccess) {
                    rq->status = BBFMM_ERR_HIP;
                    rq->error = hipGetErrorString(q);
                }
            }
            s.batch.clear();
            s.busy = false;
            s.entry->busy = false;
            s.entry = nullptr;
            cv_done.notify_all();
        }
    }

    // An idle cached entry for (model, R), or a new one if the budget allows
    // after evicting idle entries (least recently used first).  Returns
    // nullptr when the batch must wait; sets *reject when it can never fit.
    Entry *acquire(int mdl, int R, hipStream_t stream, bool *reject) {
        *reject = false;
        for (auto &e : cache)
            if (!e->busy && e->model == mdl && e->R == R) return e.get();
        const auto key = std::make_pair(mdl, R);
        auto known = need.find(key);
        if (known != need.end()) {
            if (known->second > budget) {
                *reject = true;
                return nullptr;
            }
            int64_t idle = 0;
            for (auto &e : cache)
                if (!e->busy) idle += e->bytes;
            if (in_use - idle + known->second > budget) return nullptr;   // wait for a retirement
        }
        const Model &m = models[mdl];
        bbfmm_plan_options opt{};
        opt.m2l_split = kServeSplit;
        opt.p2p_mfma = R == 1 ? 1 : 2;
        struct PlanDel {
            void operator()(Plan *q) const { plan_destroy(q); }
        };
        MemScope scope(&m.ops->hook, stream);
        std::unique_ptr<Plan, PlanDel> plan(plan_create_impl(m.tree, m.ops, R, &opt, stream));
        const int64_t bytes = plan_workspace_bytes(plan.get()) +
                              (m.tree->n_in() + m.tree->n_out()) * R * int64_t(sizeof(float));
        need[key] = bytes;
        if (bytes > budget) {
            *reject = true;
            return nullptr;
        }
        while (in_use + bytes > budget) {
            size_t victim = cache.size();
            for (size_t q = 0; q < cache.size(); ++q)
                if (!cache[q]->busy && (victim == cache.size() || cache[q]->last_use < cache[victim]->last_use))
                    victim = q;
            if (victim == cache.size()) return nullptr;     // everything cached is running
            in_use -= cache[victim]->bytes;
            cache.erase(cache.begin() + victim);
            ++st.plans_evicted;
        }
        std::unique_ptr<Entry> e(new Entry());
        e->model = mdl;
        e->R = R;
        e->sig.alloc(m.tree->n_in() * R);
        e->phi.alloc(m.tree->n_out() * R);
        plan_set_graph(plan.get(), true);
        e->plan = plan.release();
        e->bytes = bytes;
        in_use += bytes;
        ++st.plans_created;
        st.bytes_peak = std::max(st.bytes_peak, in_use);
        cache.push_back(std::move(e));
        return cache.back().get();
    }

    // Launch the batch on slot k; called with mu held.  Returns false when
    // the batch does not fit the budget right now.
    bool launch(size_t k, std::vector<Request *> &batch, int R) {
        Slot &s = slots[k];
        const int mdl = batch.front()->model;
        bool reject = false;
        Entry *e = acquire(mdl, R, s.stream, &reject);
        if (reject) {
            for (Request *rq : batch) {
                rq->status = BBFMM_ERR_BUDGET;
                rq->error = "request does not fit the HBM budget";
                rq->done = true;
                ++st.requests_done;
                rq->t_admit = rq->t_done = now_s();
            }
            cv_done.notify_all();
            return true;     // consumed (rejected)
        }
        if (e == nullptr) return false;
        const int64_t n_in = models[mdl].tree->n_in(), n_out = models[mdl].tree->n_out();
        const double t = now_s();
        int c0 = 0;
        for (Request *rq : batch) {
            k_pack<<<grid(n_in * rq->r), kThreads, 0, s.stream>>>(rq->sigma, n_in, int(rq->r), e->sig.p, R, c0);
            c0 += int(rq->r);
        }
        if (c0 < R) k_zero_cols<<<grid(n_in * (R - c0)), kThreads, 0, s.stream>>>(n_in, e->sig.p, R, c0);
        BB_LAUNCH_CHECK();
        plan_execute_impl(e->plan, e->sig.p, e->phi.p, s.stream);
        c0 = 0;
        for (Request *rq : batch) {
            k_unpack<<<grid(n_out * rq->r), kThreads, 0, s.stream>>>(e->phi.p, n_out, R, c0, rq->phi, int(rq->r));
            c0 += int(rq->r);
            rq->t_admit = t;
            rq->slot = int(k);
        }
        BB_LAUNCH_CHECK();
        for (Request *rq : batch) rq->batch_r = c0;
        BB_HIP(hipEventRecord(s.done, s.stream));
        ++st.batches;
        e->busy = true;
        e->last_use = ++tick;
        s.entry = e;
        s.batch = batch;
        s.busy = true;
        return true;
    }

    void loop() {
        if (hipSetDevice(device) != hipSuccess) {
            std::lock_guard<std::mutex> lk(mu);
            fatal = "hipSetDevice failed in the scheduler";
            return;
        }
        std::unique_lock<std::mutex> lk(mu);
        while (!stop) {
            retire();
            bool progressed = false;
            int pick = -1;
            for (size_t k = 0; k < slots.size(); ++k)
                if (!slots[k].busy) { pick = int(k); break; }
            if (!pending.empty() && pick >= 0) {
                // batch: the oldest request and later ones of the same model
                const int mdl = pending.front()->model;
                std::vector<Request *> batch;
                int64_t tot = 0;
                for (Request *rq : pending) {
                    if (rq->model != mdl) continue;
                    if (tot + rq->r > r_max) break;
                    batch.push_back(rq);
                    tot += rq->r;
                }
                int R = 1;
                while (R < tot) R *= 2;
                if (!batch.empty()) {
                    bool ok = false;
                    try {
                        ok = launch(size_t(pick), batch, R);
                    } catch (const Exception &) {
                        const std::string msg = bbfmm_last_error();
                        for (Request *rq : batch) {
                            rq->status = BBFMM_ERR_HIP;
                            rq->error = msg;
                            rq->done = true;
                        }
                        cv_done.notify_all();
                        ok = true;
                    }
                    if (ok) {
                        for (Request *rq : batch)
                            for (auto it = pending.begin(); it != pending.end(); ++it)
                                if (*it == rq) { pending.erase(it); break; }
                        progressed = true;
                    }
                }
            }
            if (!progressed) {
                bool any_busy = false;
                for (Slot &s : slots) any_busy |= s.busy;
                if (any_busy)
                    cv_work.wait_for(lk, std::chrono::microseconds(50));
                else
                    cv_work.wait(lk, [&] { return stop || !pending.empty(); });
            }
        }
    }
};

}  // namespace bbfmm

struct bbfmm_server {
    std::unique_ptr<bbfmm::Server> impl;
};

using namespace bbfmm;

extern "C" {

bbfmm_status bbfmm_server_create(int64_t hbm_budget_bytes, int32_t max_inflight, int32_t r_max,
                                 bbfmm_server **out) {
    bbfmm::clear_error();
    try {
        BB_REQUIRE(out != nullptr, "out is NULL");
        *out = nullptr;
        BB_REQUIRE(hbm_budget_bytes > 0, "hbm_budget_bytes must be positive");
        BB_REQUIRE(max_inflight >= 1 && max_inflight <= 64, "max_inflight must be in [1, 64]");
        BB_REQUIRE(r_max >= 1 && r_max <= 4096, "r_max must be in [1, 4096]");
        std::unique_ptr<bbfmm_server> sv(new bbfmm_server());
        sv->impl.reset(new Server());
        Server &s = *sv->impl;
        s.budget = hbm_budget_bytes;
        s.max_inflight = max_inflight;
        s.r_max = r_max;
        BB_HIP(hipGetDevice(&s.device));
        s.slots.resize(max_inflight);
        for (Slot &sl : s.slots) {
            BB_HIP(hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking));
            BB_HIP(hipEventCreateWithFlags(&sl.done, hipEventDisableTiming));
        }
        s.worker = std::thread([&s] { s.loop(); });
        *out = sv.release();
        return BBFMM_OK;
    } catch (const Exception &e) {
        return e.status;
    } catch (...) {
        return BBFMM_ERR_INTERNAL;
    }
}

bbfmm_status bbfmm_server_add(bbfmm_server *sv, const bbfmm_tree *tree, const bbfmm_ops *ops,
                              int32_t *model_id) {
    bbfmm::clear_error();
    try {
        BB_REQUIRE(sv && tree && ops && model_id, "NULL argument");
        BB_REQUIRE(ops->tree == tree, "operators were built for another tree");
        Server &s = *sv->impl;
        std::lock_guard<std::mutex> lk(s.mu);
        s.models.push_back(Model{tree, ops});
        *model_id = int32_t(s.models.size() - 1);
        return BBFMM_OK;
    } catch (const Exception &e) {
        return e.status;
    }
}

bbfmm_status bbfmm_server_submit(bbfmm_server *sv, int32_t model_id, const float *sigma, int64_t r,
                                 float *phi, uint64_t *request_id) {
    bbfmm::clear_error();
    try {
        BB_REQUIRE(sv && sigma && phi && request_id, "NULL argument");
        Server &s = *sv->impl;
        std::lock_guard<std::mutex> lk(s.mu);
        BB_REQUIRE(s.fatal.empty(), "%s", s.fatal.c_str());
        BB_REQUIRE(model_id >= 0 && model_id < int32_t(s.models.size()), "unknown model %d", model_id);
        BB_REQUIRE(r >= 1 && r <= s.r_max, "r must be in [1, r_max]");
        for (const void *ptr : {static_cast<const void *>(sigma), static_cast<const void *>(phi)}) {
            hipPointerAttribute_t attr{};
            BB_REQUIRE(hipPointerGetAttributes(&attr, ptr) == hipSuccess &&
                           (attr.type == hipMemoryTypeDevice || attr.type == hipMemoryTypeManaged),
                       "sigma / phi must be device pointers");
        }
        std::unique_ptr<Request> rq(new Request());
        rq->id = s.next_id++;
        rq->model = model_id;
        rq->sigma = sigma;
        rq->phi = phi;
        rq->r = r;
        rq->t_submit = now_s();
        *request_id = rq->id;
        s.pending.push_back(rq.get());
        s.requests[rq->id] = std::move(rq);
        s.cv_work.notify_all();
        return BBFMM_OK;
    } catch (const Exception &e) {
        return e.status;
    }
}

bbfmm_status bbfmm_server_wait(bbfmm_server *sv, uint64_t request_id, bbfmm_request_stats *stats) {
    bbfmm::clear_error();
    try {
        BB_REQUIRE(sv != nullptr, "server is NULL");
        Server &s = *sv->impl;
        std::unique_lock<std::mutex> lk(s.mu);
        auto it = s.requests.find(request_id);
        if (it == s.requests.end()) fail(BBFMM_ERR_NOT_FOUND, "unknown request %llu", (unsigned long long)request_id);
        Request *rq = it->second.get();
        ++s.waiters;
        s.cv_done.wait(lk, [&] { return rq->done || !s.fatal.empty(); });
        --s.waiters;
        s.cv_done.notify_all();            // a destroy may be waiting for the waiters
        BB_REQUIRE(rq->done, "%s", s.fatal.c_str());
        if (stats) {
            stats->t_submit = rq->t_submit;
            stats->t_admit = rq->t_admit;
            stats->t_done = rq->t_done;
            stats->batch_r = rq->batch_r;
            stats->slot = rq->slot;
        }
        const bbfmm_status st = rq->status;
        const std::string err = rq->error;
        s.requests.erase(request_id);      // `it` may be stale: submits rehash the map
        if (st != BBFMM_OK) fail(st, "%s", err.c_str());
        return BBFMM_OK;
    } catch (const Exception &e) {
        return e.status;
    }
}

bbfmm_status bbfmm_server_cancel(bbfmm_server *sv, uint64_t request_id) {
    bbfmm::clear_error();
    try {
        BB_REQUIRE(sv != nullptr, "server is NULL");
        Server &s = *sv->impl;
        std::lock_guard<std::mutex> lk(s.mu);
        auto it = s.requests.find(request_id);
        if (it == s.requests.end()) fail(BBFMM_ERR_NOT_FOUND, "unknown request %llu", (unsigned long long)request_id);
        Request *rq = it->second.get();
        for (auto p = s.pending.begin(); p != s.pending.end(); ++p)
            if (*p == rq) {
                s.pending.erase(p);
                rq->status = BBFMM_ERR_CANCELLED;
                rq->error = "cancelled";
                rq->done = true;
                rq->t_admit = rq->t_done = now_s();
                ++s.st.requests_done;
                s.cv_done.notify_all();
                return BBFMM_OK;
            }
        fail(BBFMM_ERR_INVALID_ARG, "request %llu was already admitted (or is complete)",
             (unsigned long long)request_id);
    } catch (const Exception &e) {
        return e.status;
    }
}

bbfmm_status bbfmm_server_get_stats(bbfmm_server *sv, bbfmm_server_stats *out) {
    bbfmm::clear_error();
    try {
        BB_REQUIRE(sv != nullptr && out != nullptr, "NULL argument");
        Server &s = *sv->impl;
        std::lock_guard<std::mutex> lk(s.mu);
        *out = s.st;
        out->bytes_in_use = s.in_use;
        return BBFMM_OK;
    } catch (const Exception &e) {
        return e.status;
    }
}

bbfmm_status bbfmm_server_destroy(bbfmm_server *sv) {
    bbfmm::clear_error();
    delete sv;
    return BBFMM_OK;
}

}  // extern "C"
