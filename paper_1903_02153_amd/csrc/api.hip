// C-ABI entry points of libbbfmm (declared in include/bbfmm.h).
// Each entry point converts internal exceptions into a bbfmm_status and a
// thread-local message; nothing propagates across the ABI.
#include <algorithm>
#include <cstring>
#include <vector>
#include <mutex>
#include <new>

#include "common.h"

namespace bbfmm {

namespace {
thread_local char g_err[1024] = "";
}

void fail(bbfmm_status st, const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
    throw Exception{st};
}

void clear_error() { g_err[0] = '\0'; }

template <class F>
bbfmm_status guarded(F &&f) {
    clear_error();
    try {
        f();
        return BBFMM_OK;
    } catch (const Exception &e) {
        return e.status;
    } catch (const std::bad_alloc &) {
        snprintf(g_err, sizeof(g_err), "host allocation failed");
        return BBFMM_ERR_OUT_OF_MEMORY;
    } catch (...) {
        snprintf(g_err, sizeof(g_err), "unexpected internal error");
        return BBFMM_ERR_INTERNAL;
    }
}

const char *last_error() { return g_err; }

// ------------------------------------------------------ device memory ----
namespace {
thread_local MemSource g_mem;
Counters g_counters;
std::mutex g_pool_mu;
std::vector<std::pair<int, hipStream_t>> g_side_pool;   // (device, idle stream)
}  // namespace

MemSource &current_mem() { return g_mem; }

MemScope::MemScope(const bbfmm_allocator *hook, hipStream_t stream) : saved(g_mem) {
    g_mem.hook = hook ? *hook : bbfmm_allocator{};
    g_mem.stream = stream;
}
MemScope::~MemScope() { g_mem = saved; }

void *device_alloc(size_t bytes, const MemSource &src) {
    void *p = nullptr;
    if (src.hook.alloc) {
        p = src.hook.alloc(bytes, src.stream, src.hook.ctx);
        if (p == nullptr)
            fail(BBFMM_ERR_OUT_OF_MEMORY, "the allocator hook returned NULL for %zu bytes", bytes);
    } else {
        BB_HIP(hipMalloc(&p, bytes));
    }
    ++g_counters.buffers;
    g_counters.bytes += int64_t(bytes);
    return p;
}

void device_free(void *p, size_t bytes, const MemSource &src) {
    if (src.hook.alloc) {
        if (src.hook.free) src.hook.free(p, src.stream, src.hook.ctx);
    } else {
        (void)hipFree(p);
    }
    --g_counters.buffers;
    g_counters.bytes -= int64_t(bytes);
}

Counters &counters() { return g_counters; }

hipEvent_t make_event(unsigned flags) {
    hipEvent_t e = nullptr;
    BB_HIP(hipEventCreateWithFlags(&e, flags));
    ++g_counters.events;
    return e;
}
void destroy_event(hipEvent_t e) {
    if (!e) return;
    (void)hipEventDestroy(e);
    --g_counters.events;
}
hipStream_t make_stream() {
    hipStream_t s = nullptr;
    BB_HIP(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
    ++g_counters.streams;
    return s;
}
void destroy_stream(hipStream_t s) {
    if (!s) return;
    (void)hipStreamDestroy(s);
    --g_counters.streams;
}

hipStream_t acquire_side_stream() {
    int dev = 0;
    BB_HIP(hipGetDevice(&dev));
    {
        std::lock_guard<std::mutex> lk(g_pool_mu);
        for (size_t i = 0; i < g_side_pool.size(); ++i)
            if (g_side_pool[i].first == dev) {
                hipStream_t s = g_side_pool[i].second;
                g_side_pool.erase(g_side_pool.begin() + long(i));
                return s;
            }
    }
    return make_stream();
}

void release_side_stream(hipStream_t s) {
    if (!s) return;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return;
    std::lock_guard<std::mutex> lk(g_pool_mu);
    g_side_pool.emplace_back(dev, s);
}

template <class T>
void copy_out(const T *dev, int64_t count, void *dst, int64_t capacity, int64_t *size) {
    const int64_t bytes = count * int64_t(sizeof(T));
    if (size) *size = bytes;
    if (dst == nullptr) return;
    BB_REQUIRE(capacity >= bytes, "destination holds %lld bytes, %lld needed",
               (long long)capacity, (long long)bytes);
    if (bytes > 0) BB_HIP(hipMemcpy(dst, dev, size_t(bytes), hipMemcpyDeviceToHost));
}

}  // namespace bbfmm

using namespace bbfmm;

struct bbfmm_plan {
    Plan *impl = nullptr;
    bbfmm_plan_options asked{};        // the options the plan was created with
    ~bbfmm_plan() { plan_destroy(impl); }
};

extern "C" {

const char *bbfmm_last_error(void) { return last_error(); }

bbfmm_status bbfmm_build_tree(const float *points, int64_t n, const bbfmm_tree_params *params,
                              const bbfmm_allocator *allocator, void *stream, bbfmm_tree **out) {
    return guarded([&] {
        BB_REQUIRE(params != nullptr && out != nullptr, "params / out is NULL");
        *out = nullptr;
        BB_REQUIRE(allocator == nullptr || (allocator->alloc && allocator->free),
                   "allocator needs both alloc and free");
        hipStream_t s = static_cast<hipStream_t>(stream);
        MemScope scope(allocator, s);
        *out = build_tree_impl(points, n, *params, s);
        if (allocator) (*out)->hook = *allocator;
    });
}

bbfmm_status bbfmm_build_tree_sets(const float *targets, int64_t n_targets, const float *sources,
                                   int64_t n_sources, const bbfmm_tree_params *params,
                                   const bbfmm_allocator *allocator, void *stream,
                                   bbfmm_tree **out) {
    return guarded([&] {
        BB_REQUIRE(params != nullptr && out != nullptr, "params / out is NULL");
        *out = nullptr;
        BB_REQUIRE(allocator == nullptr || (allocator->alloc && allocator->free),
                   "allocator needs both alloc and free");
        hipStream_t s = static_cast<hipStream_t>(stream);
        MemScope scope(allocator, s);
        *out = build_tree_sets_impl(targets, n_targets, sources, n_sources, *params, s);
        if (allocator) (*out)->hook = *allocator;
    });
}

bbfmm_status bbfmm_tree_info_get(const bbfmm_tree *t, bbfmm_tree_info *out) {
    return guarded([&] {
        BB_REQUIRE(t != nullptr && out != nullptr, "tree / out is NULL");
        std::memset(out, 0, sizeof(*out));
        out->n_points = t->n;
        out->depth = t->depth;
        out->cheb_order = t->params.cheb_order;
        out->kernel_id = t->params.kernel_id;
        out->kernel_param = t->params.kernel_param;
        for (int d = 0; d < 3; ++d) out->lo[d] = t->lo[d];
        out->side = t->side;
        out->scale = t->scale;
        out->max_leaf_points = t->max_leaf;
        for (int l = 0; l < t->depth; ++l) {
            out->cells[l] = t->lv[l].C;
            out->pairs[l] = t->lv[l].npairs;
        }
        out->near_pairs = t->near_pairs;
        out->n_targets = t->n_out();
        out->n_sources = t->n_in();
        out->adaptive = t->adaptive ? 1 : 0;
        out->n_leaves = t->leaves().C;
        out->w_entries = t->w_nnz;
    });
}

bbfmm_status bbfmm_tree_export(const bbfmm_tree *t, int32_t what, int32_t level, void *dst,
                               int64_t capacity, int64_t *size) {
    return guarded([&] {
        BB_REQUIRE(t != nullptr, "tree is NULL");
        const bool per_level = (what >= BBFMM_TA_KEYS && what <= BBFMM_TA_CE) ||
                               what == BBFMM_TA_X_OFF || what == BBFMM_TA_X_LEAF;
        const bool pair = what >= BBFMM_TA_PAIR_T && what <= BBFMM_TA_PAIR_GOFF;
        if (per_level || pair) {
            if (level < 0 || level >= t->depth || (pair && level < 2))
                fail(BBFMM_ERR_NOT_FOUND, "level %d has no such array", level);
        }
        const bool adaptive_only = what >= BBFMM_TA_W_OFF && what <= BBFMM_TA_X_LEAF;
        if (adaptive_only && !t->adaptive)
            fail(BBFMM_ERR_NOT_FOUND, "tree array %d exists on level-adaptive trees only", what);
        const LevelData *lv = (per_level || pair) ? &t->lv[level] : nullptr;
        const int64_t NL = t->leaves().C;
        switch (what) {
        case BBFMM_TA_PERM: copy_out(t->perm.p, t->n, dst, capacity, size); break;
        case BBFMM_TA_KEYS: copy_out(lv->keys.p, lv->C, dst, capacity, size); break;
        case BBFMM_TA_PB: copy_out(lv->pb.p, lv->C, dst, capacity, size); break;
        case BBFMM_TA_PE: copy_out(lv->pe.p, lv->C, dst, capacity, size); break;
        case BBFMM_TA_PARENT: copy_out(lv->parent.p, lv->C, dst, capacity, size); break;
        case BBFMM_TA_CB: copy_out(lv->cb.p, lv->C, dst, capacity, size); break;
        case BBFMM_TA_CE: copy_out(lv->ce.p, lv->C, dst, capacity, size); break;
        case BBFMM_TA_NBR_OFF: copy_out(t->nbr_off.p, NL + 1, dst, capacity, size); break;
        case BBFMM_TA_NBR_IDX: copy_out(t->nbr_idx.p, t->nbr_nnz, dst, capacity, size); break;
        case BBFMM_TA_PAIR_T: copy_out(lv->pair_t.p, lv->npairs, dst, capacity, size); break;
        case BBFMM_TA_PAIR_TGT: copy_out(lv->pair_tgt.p, lv->npairs, dst, capacity, size); break;
        case BBFMM_TA_PAIR_SRC: copy_out(lv->pair_src.p, lv->npairs, dst, capacity, size); break;
        case BBFMM_TA_PAIR_GOFF: copy_out(lv->pair_goff.p, int64_t(kNumT) + 1, dst, capacity, size); break;
        case BBFMM_TA_LEAF_LEVEL: copy_out(t->fl_level.p, NL, dst, capacity, size); break;
        case BBFMM_TA_LEAF_CELL: copy_out(t->fl_cell.p, NL, dst, capacity, size); break;
        case BBFMM_TA_W_OFF: copy_out(t->w_off.p, NL + 1, dst, capacity, size); break;
        case BBFMM_TA_W_LEVEL: copy_out(t->w_level.p, t->w_nnz, dst, capacity, size); break;
        case BBFMM_TA_W_CELL: copy_out(t->w_cell.p, t->w_nnz, dst, capacity, size); break;
        case BBFMM_TA_X_OFF: copy_out(lv->x_off.p, int64_t(lv->C) + 1, dst, capacity, size); break;
        case BBFMM_TA_X_LEAF: {
            int32_t nx = 0;
            if (lv->C > 0)
                BB_HIP(hipMemcpy(&nx, lv->x_off.p + lv->C, sizeof(int32_t), hipMemcpyDeviceToHost));
            copy_out(lv->x_leaf.p, nx, dst, capacity, size);
            break;
        }
        default: fail(BBFMM_ERR_NOT_FOUND, "unknown tree array %d", what);
        }
    });
}

bbfmm_status bbfmm_precompute_operators(const bbfmm_tree *t, double svd_eps, int32_t precision,
                                        const bbfmm_allocator *allocator, void *stream,
                                        bbfmm_ops **out) {
    return guarded([&] {
        BB_REQUIRE(out != nullptr, "out is NULL");
        *out = nullptr;
        precompute_check(svd_eps, precision);
        BB_REQUIRE(t != nullptr, "tree is NULL");
        BB_REQUIRE(allocator == nullptr || (allocator->alloc && allocator->free),
                   "allocator needs both alloc and free");
        const bbfmm_allocator hook = allocator ? *allocator : t->hook;
        hipStream_t s = static_cast<hipStream_t>(stream);
        MemScope scope(&hook, s);
        *out = precompute_impl(t, svd_eps, precision, s);
        (*out)->hook = hook;
    });
}

bbfmm_status bbfmm_ops_rank(const bbfmm_ops *o, int32_t level, int32_t *k) {
    return guarded([&] {
        BB_REQUIRE(o != nullptr && k != nullptr, "ops / k is NULL");
        if (level < 2 || level >= o->tree->depth || o->lv[level].set == nullptr)
            fail(BBFMM_ERR_NOT_FOUND, "level %d has no M2L operators", level);
        *k = o->lv[level].set->k;
    });
}

bbfmm_status bbfmm_ops_export(const bbfmm_ops *o, int32_t what, int32_t level, void *dst,
                              int64_t capacity, int64_t *size) {
    return guarded([&] {
        BB_REQUIRE(o != nullptr, "ops is NULL");
        if (level < 2 || level >= o->tree->depth || o->lv[level].set == nullptr)
            fail(BBFMM_ERR_NOT_FOUND, "level %d has no M2L operators", level);
        const OpSet &set = *o->lv[level].set;
        const int64_t m = o->m, k = set.k;
        if (o->precision == BBFMM_M2L_FFT)
            fail(BBFMM_ERR_NOT_FOUND, "the FFT M2L keeps operator spectra, not U, V, C");
        switch (what) {
        case BBFMM_OA_U: copy_out(set.U64.p, m * k, dst, capacity, size); break;
        case BBFMM_OA_V: copy_out(set.V64.p, m * k, dst, capacity, size); break;
        case BBFMM_OA_C: {
            copy_out(set.C64.p, int64_t(kNumT) * k * k, dst, capacity, size);
            if (dst != nullptr && o->lv[level].scale != 1.0) {
                double *d = static_cast<double *>(dst);
                for (int64_t i = 0; i < int64_t(kNumT) * k * k; ++i) d[i] *= o->lv[level].scale;
            }
            break;
        }
        case BBFMM_OA_SV_FAT:
            if (set.sv_fat.n == 0) fail(BBFMM_ERR_NOT_FOUND, "no singular values (imported or eps = 0)");
            copy_out(set.sv_fat.p, m, dst, capacity, size);
            break;
        case BBFMM_OA_SV_THIN:
            if (set.sv_thin.n == 0) fail(BBFMM_ERR_NOT_FOUND, "no singular values (imported or eps = 0)");
            copy_out(set.sv_thin.p, m, dst, capacity, size);
            break;
        default: fail(BBFMM_ERR_NOT_FOUND, "unknown operator array %d", what);
        }
    });
}

bbfmm_status bbfmm_ops_import(const bbfmm_tree *t, int32_t precision, const int32_t *ranks,
                              const double *U, const double *V, const double *C, void *stream,
                              bbfmm_ops **out) {
    return guarded([&] {
        BB_REQUIRE(t != nullptr && out != nullptr, "tree / out is NULL");
        *out = nullptr;
        BB_REQUIRE(precision == BBFMM_M2L_FP32 || precision == BBFMM_M2L_BF16X3 ||
                       precision == BBFMM_M2L_FP16_SCALED,
                   "unsupported M2L precision %d", precision);
        hipStream_t s = static_cast<hipStream_t>(stream);
        MemScope scope(&t->hook, s);
        std::unique_ptr<bbfmm_ops> ops(new bbfmm_ops());
        ops->tree = t;
        ops->hook = t->hook;
        ops->n = t->params.cheb_order;
        ops->m = ops->n * ops->n * ops->n;
        ops->mp = int(ceil_div(ops->m, 16) * 16);
        ops->precision = precision;
        cheb_setup(ops.get(), s);
        const int L = t->leaf_level();
        if (L >= 2) BB_REQUIRE(ranks && U && V && C, "ranks / U / V / C is NULL");
        const int64_t m = ops->m;
        int64_t offUV = 0, offC = 0;
        for (int lvl = 2; lvl <= L; ++lvl) {
            const int k = ranks[lvl];
            BB_REQUIRE(k >= 1 && k <= m, "rank %d of level %d outside [1, %lld]", k, lvl, (long long)m);
            std::unique_ptr<OpSet> set(new OpSet());
            set->k = k;
            set->U64.alloc(m * k);
            set->V64.alloc(m * k);
            set->C64.alloc(int64_t(kNumT) * k * k);
            BB_HIP(hipMemcpy(set->U64.p, U + offUV, m * k * sizeof(double), hipMemcpyHostToDevice));
            BB_HIP(hipMemcpy(set->V64.p, V + offUV, m * k * sizeof(double), hipMemcpyHostToDevice));
            BB_HIP(hipMemcpy(set->C64.p, C + offC, int64_t(kNumT) * k * k * sizeof(double),
                             hipMemcpyHostToDevice));
            offUV += m * k;
            offC += int64_t(kNumT) * k * k;
            finalize_opset(*set, int(m), ops->mp, precision, s);
            ops->lv[lvl].set = set.get();
            ops->lv[lvl].scale = 1.0;
            ops->sets.push_back(std::move(set));
        }
        *out = ops.release();
    });
}

bbfmm_status bbfmm_plan_create_ex(const bbfmm_tree *t, const bbfmm_ops *o, int64_t r,
                                  const bbfmm_plan_options *opt, const bbfmm_allocator *allocator,
                                  void *stream, bbfmm_plan **out) {
    return guarded([&] {
        BB_REQUIRE(out != nullptr, "out is NULL");
        *out = nullptr;
        BB_REQUIRE(allocator == nullptr || (allocator->alloc && allocator->free),
                   "allocator needs both alloc and free");
        hipStream_t s = static_cast<hipStream_t>(stream);
        // (options, tree and operators are validated by plan_create_impl first)
        MemScope scope(allocator ? allocator : (o ? &o->hook : nullptr), s);
        std::unique_ptr<bbfmm_plan> p(new bbfmm_plan());
        p->impl = plan_create_impl(t, o, r, opt, s);
        if (opt) p->asked = *opt;
        *out = p.release();
    });
}

bbfmm_status bbfmm_plan_create(const bbfmm_tree *t, const bbfmm_ops *o, int64_t r,
                               bbfmm_plan **out) {
    return bbfmm_plan_create_ex(t, o, r, nullptr, nullptr, nullptr, out);
}

bbfmm_status bbfmm_plan_execute(bbfmm_plan *p, const float *sigma, float *phi, void *stream) {
    return guarded([&] {
        BB_REQUIRE(p != nullptr, "plan is NULL");
        plan_execute_impl(p->impl, sigma, phi, static_cast<hipStream_t>(stream));
    });
}

bbfmm_status bbfmm_plan_get_options(const bbfmm_plan *p, bbfmm_plan_options *out) {
    return guarded([&] {
        BB_REQUIRE(p != nullptr && out != nullptr, "plan / out is NULL");
        *out = p->asked;
        plan_resolved_options(p->impl, out);
    });
}

bbfmm_status bbfmm_plan_workspace_bytes(const bbfmm_plan *p, int64_t *bytes) {
    return guarded([&] {
        BB_REQUIRE(p != nullptr && bytes != nullptr, "plan / bytes is NULL");
        *bytes = plan_workspace_bytes(p->impl);
    });
}

bbfmm_status bbfmm_plan_set_timing(bbfmm_plan *p, int32_t enable) {
    return guarded([&] {
        BB_REQUIRE(p != nullptr, "plan is NULL");
        plan_set_timing(p->impl, enable != 0);
    });
}

bbfmm_status bbfmm_plan_set_graph(bbfmm_plan *p, int32_t enable) {
    return guarded([&] {
        BB_REQUIRE(p != nullptr, "plan is NULL");
        plan_set_graph(p->impl, enable != 0);
    });
}

bbfmm_status bbfmm_plan_stage_times(bbfmm_plan *p, double *ms, int64_t *executions,
                                    int32_t reset) {
    return guarded([&] {
        BB_REQUIRE(p != nullptr, "plan is NULL");
        plan_stage_times(p->impl, ms, executions, reset != 0);
    });
}

namespace {

bool is_device_ptr(const void *ptr) {
    hipPointerAttribute_t attr{};
    return ptr != nullptr && hipPointerGetAttributes(&attr, ptr) == hipSuccess &&
           (attr.type == hipMemoryTypeDevice || attr.type == hipMemoryTypeManaged);
}

// median milliseconds of `reps` products with these options (after one untimed)
double time_options(const bbfmm_tree *t, const bbfmm_ops *o, int64_t r, const bbfmm_plan_options &op,
                    const float *sigma, float *phi, hipStream_t s, int reps) {
    MemScope scope(&o->hook, s);
    std::unique_ptr<bbfmm_plan> p(new bbfmm_plan());
    p->impl = plan_create_impl(t, o, r, &op, s);
    plan_execute_impl(p->impl, sigma, phi, s);
    std::vector<hipEvent_t> ev(size_t(2 * reps), nullptr);
    struct Events {
        std::vector<hipEvent_t> &e;
        ~Events() {
            for (hipEvent_t x : e)
                destroy_event(x);
        }
    } guard{ev};
    for (hipEvent_t &e : ev) e = make_event(hipEventDefault);
    for (int i = 0; i < reps; ++i) {
        BB_HIP(hipEventRecord(ev[2 * i], s));
        plan_execute_impl(p->impl, sigma, phi, s);
        BB_HIP(hipEventRecord(ev[2 * i + 1], s));
    }
    BB_HIP(hipEventSynchronize(ev.back()));
    std::vector<float> ms(static_cast<size_t>(reps));
    for (int i = 0; i < reps; ++i) BB_HIP(hipEventElapsedTime(&ms[i], ev[2 * i], ev[2 * i + 1]));
    std::sort(ms.begin(), ms.end());
    BB_HIP(hipStreamSynchronize(s));    // the workspace is released after the stream used it
    return ms[size_t(reps / 2)];
}

}  // namespace

bbfmm_status bbfmm_plan_autotune(const bbfmm_tree *t, const bbfmm_ops *o, int64_t r,
                                 const float *sigma, float *phi, void *stream, int32_t reps,
                                 bbfmm_plan_options *best, double *best_ms) {
    return guarded([&] {
        BB_REQUIRE(t != nullptr && o != nullptr && best != nullptr, "NULL argument");
        BB_REQUIRE(reps >= 1 && reps <= 100, "reps must be in [1, 100]");
        BB_REQUIRE(is_device_ptr(sigma) && is_device_ptr(phi), "sigma / phi must be device pointers");
        hipStream_t s = static_cast<hipStream_t>(stream);
        bbfmm_plan_options cur{};
        double cur_ms = time_options(t, o, r, cur, sigma, phi, s, reps);   // the heuristic
        auto consider = [&](const bbfmm_plan_options &c) {
            const double ms = time_options(t, o, r, c, sigma, phi, s, reps);
            if (ms < cur_ms) {
                cur_ms = ms;
                cur = c;
            }
        };
        for (int split : {1, 2, 3, 4, 8}) {
            bbfmm_plan_options c = cur;
            c.m2l_split = split;
            consider(c);
        }
        for (int path = 1; path <= 2; ++path) {
            bbfmm_plan_options c = cur;
            c.p2p_mfma = path;
            consider(c);
        }
        if (cur.p2p_mfma != 2)
            for (int cap : {4, 8, 16}) {
                bbfmm_plan_options c = cur;
                c.p2p_mfma = 1;
                c.p2p_max_split = cap;
                consider(c);
            }
        for (int ov = 1; ov <= 2; ++ov) {
            bbfmm_plan_options c = cur;
            c.overlap = ov;
            consider(c);
        }
        if (r == 1 && cur.p2p_mfma != 2)
            for (int pk = 1; pk <= 2; ++pk) {
                bbfmm_plan_options c = cur;
                c.p2p_mfma = 1;
                c.p2p_pack = pk;
                consider(c);
            }
        if (cur.overlap != 1 && cur.p2p_mfma != 2)
            for (int nw : {512, 1024, 2048, 4096}) {
                bbfmm_plan_options c = cur;
                c.p2p_mfma = 1;
                c.p2p_waves = nw;
                consider(c);
            }
        if (o->precision == BBFMM_M2L_FP32) {
            bbfmm_plan_options c = cur;
            c.m2l_layout = 2;
            consider(c);
        }
        for (int xc = 1; xc <= 2; ++xc) {
            bbfmm_plan_options c = cur;
            c.m2l_xcd = xc;
            consider(c);
        }
        if (r >= 4)
            for (int lf = 1; lf <= 2; ++lf) {
                bbfmm_plan_options c = cur;
                c.leaf_fused = lf;
                consider(c);
            }
        if (cur.overlap != 1)
            for (int occ : {3, 2}) {
                bbfmm_plan_options c = cur;
                c.m2l_occupancy = occ;
                consider(c);
            }
        for (int sch = 1; sch <= 2; ++sch) {
            bbfmm_plan_options c = cur;
            c.m2l_schedule = sch;
            consider(c);
        }
        if (o->precision == BBFMM_M2L_BF16X3 || o->precision == BBFMM_M2L_FP16_SCALED)
            for (int blk = 1; blk <= 2; ++blk) {
                bbfmm_plan_options c = cur;
                c.m2l_block = blk;
                consider(c);
            }
        if ((o->precision == BBFMM_M2L_BF16X3 || o->precision == BBFMM_M2L_FP16_SCALED) &&
            cur.m2l_block != 1 && r > 16)
            for (int rt : {16, 32, 64}) {
                if (rt > 16 && rt / 2 >= r) continue;      // wider than the block of columns
                bbfmm_plan_options c = cur;
                c.m2l_block = 2;
                c.m2l_rtile = rt;
                consider(c);
            }
        if ((o->precision == BBFMM_M2L_BF16X3 || o->precision == BBFMM_M2L_FP16_SCALED) &&
            cur.m2l_block != 1 && r >= 32)
            for (int mf = 1; mf <= 2; ++mf) {
                bbfmm_plan_options c = cur;
                c.m2l_block = 2;
                c.m2l_mfma = mf;
                consider(c);
            }
        // make every choice explicit: what the heuristic picked for the zeros
        MemScope scope(&o->hook, s);
        std::unique_ptr<bbfmm_plan> p(new bbfmm_plan());
        p->impl = plan_create_impl(t, o, r, &cur, s);
        plan_resolved_options(p->impl, &cur);
        *best = cur;
        if (best_ms) *best_ms = cur_ms;
    });
}

bbfmm_status bbfmm_matvec(const bbfmm_tree *t, const bbfmm_ops *o, const float *sigma, int64_t r,
                          float *phi, void *stream) {
    return guarded([&] {
        BB_REQUIRE(t != nullptr && o != nullptr, "tree or ops is NULL");
        BB_REQUIRE(o->tree == t, "operators were built for another tree");
        BB_REQUIRE(sigma != nullptr && phi != nullptr, "sigma / phi is NULL");
        BB_REQUIRE(r >= 1 && r <= 4096, "r must be in [1, 4096]");
        matvec_cached(const_cast<bbfmm_ops *>(o), sigma, r, phi, static_cast<hipStream_t>(stream));
    });
}

bbfmm_status bbfmm_get_runtime_counters(bbfmm_runtime_counters *out) {
    return guarded([&] {
        BB_REQUIRE(out != nullptr, "out is NULL");
        const Counters &c = counters();
        out->device_buffers = c.buffers.load();
        out->device_bytes = c.bytes.load();
        out->plans = c.plans.load();
        out->streams = c.streams.load();
        out->events = c.events.load();
        out->plans_freed_in_flight = c.plans_freed_in_flight.load();
    });
}

void bbfmm_tree_free(bbfmm_tree *t) { delete t; }
void bbfmm_ops_free(bbfmm_ops *o) { delete o; }
void bbfmm_plan_free(bbfmm_plan *p) { delete p; }

}  // extern "C"
