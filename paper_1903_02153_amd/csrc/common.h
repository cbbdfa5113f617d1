// Internal definitions shared by the translation units of libbbfmm.
// Every host-side failure is raised as bbfmm::Exception and turned into a
// bbfmm_status at the C-ABI boundary (api.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "bbfmm.h"

namespace bbfmm {

constexpr int kQBits = 21;          // binning resolution per axis (2^21 cells)
constexpr int kMaxLevels = 22;      // levels 0..21
constexpr int kNumT = 316;          // M2L transfer vectors per level
constexpr int kSlots = 189;         // transfer vectors valid for one octant
constexpr int kMaxOrder = 8;

struct Exception {
    bbfmm_status status;
};

[[noreturn]] void fail(bbfmm_status st, const char *fmt, ...);
void clear_error();

#define BB_HIP(call)                                                            \
    do {                                                                        \
        hipError_t e_ = (call);                                                 \
        if (e_ != hipSuccess)                                                   \
            ::bbfmm::fail(e_ == hipErrorOutOfMemory ? BBFMM_ERR_OUT_OF_MEMORY   \
                                                    : BBFMM_ERR_HIP,            \
                          "%s: %s (%s:%d)", #call, hipGetErrorString(e_),       \
                          __FILE__, __LINE__);                                  \
    } while (0)

#define BB_LAUNCH_CHECK() BB_HIP(hipGetLastError())

#define BB_REQUIRE(cond, ...)                                                   \
    do {                                                                        \
        if (!(cond)) ::bbfmm::fail(BBFMM_ERR_INVALID_ARG, __VA_ARGS__);         \
    } while (0)

#define BB_INTERNAL(cond, ...)                                                  \
    do {                                                                        \
        if (!(cond)) ::bbfmm::fail(BBFMM_ERR_INTERNAL, __VA_ARGS__);            \
    } while (0)

// ------------------------------------------------------ device memory ----
// Where device memory comes from: the caller's allocator hook
// (bbfmm_allocator, e.g. a framework's caching allocator) or hipMalloc /
// hipFree.  A constructing call sets the source for its thread with a
// MemScope; every DBuf allocated meanwhile remembers the hook and stream it
// came from and returns its memory through the same hook.
struct MemSource {
    bbfmm_allocator hook{};          // hook.alloc == nullptr: hipMalloc / hipFree
    hipStream_t stream = nullptr;
};
MemSource &current_mem();            // this thread's source
struct MemScope {
    MemSource saved;
    MemScope(const bbfmm_allocator *hook, hipStream_t stream);
    ~MemScope();
    MemScope(const MemScope &) = delete;
    MemScope &operator=(const MemScope &) = delete;
};
void *device_alloc(size_t bytes, const MemSource &src);
void device_free(void *p, size_t bytes, const MemSource &src);

// Live-resource counters of the library (bbfmm_get_runtime_counters).
struct Counters {
    std::atomic<int64_t> buffers{0}, bytes{0}, plans{0}, streams{0}, events{0};
    std::atomic<int64_t> plans_freed_in_flight{0};
};
Counters &counters();
hipEvent_t make_event(unsigned flags);   // counted hipEventCreateWithFlags
void destroy_event(hipEvent_t e);        // NULL-safe
hipStream_t make_stream();               // counted non-blocking stream
void destroy_stream(hipStream_t s);      // NULL-safe
// Non-blocking streams reused across plans (one plan holds one at a time);
// streams are created on demand and kept until the process ends.
hipStream_t acquire_side_stream();
void release_side_stream(hipStream_t s);

// Owning device buffer.
template <class T>
struct DBuf {
    T *p = nullptr;
    size_t n = 0;
    MemSource src;
    DBuf() = default;
    explicit DBuf(size_t count) { alloc(count); }
    DBuf(const DBuf &) = delete;
    DBuf &operator=(const DBuf &) = delete;
    DBuf(DBuf &&o) noexcept : p(o.p), n(o.n), src(o.src) { o.p = nullptr; o.n = 0; }
    DBuf &operator=(DBuf &&o) noexcept {
        if (this != &o) { release(); p = o.p; n = o.n; src = o.src; o.p = nullptr; o.n = 0; }
        return *this;
    }
    ~DBuf() { release(); }
    void alloc(size_t count) {
        release();
        if (count == 0) return;
        src = current_mem();
        p = static_cast<T *>(device_alloc(count * sizeof(T), src));
        n = count;
    }
    void release() {
        if (p) device_free(p, n * sizeof(T), src);
        p = nullptr;
        n = 0;
    }
    size_t bytes() const { return n * sizeof(T); }
};

inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

// Host-side table of the 316 transfer vectors (compact index order) and,
// per octant, the 189 of them whose parents are adjacent.
struct TransferTables {
    int tvec[kNumT][3];
    int slot_t[8][kSlots];      // octant, slot -> compact t index
    int t_slot[8][kNumT];       // octant, t -> slot or -1
    TransferTables();
};
const TransferTables &transfer_tables();

// ---------------------------------------------------------------- tree ----
struct LevelData {
    int32_t C = 0;
    DBuf<uint64_t> keys;
    DBuf<int32_t> pb, pe, parent, cb, ce;
    // M2L structures, levels >= 2
    DBuf<int32_t> itab;             // [C][189]: source cell per slot, -1 if none
    DBuf<int32_t> oct_cells;        // cells grouped by octant, then by interaction-slot
                                    // pattern, Morton order within a group
    int32_t oct_off[9] = {0};       // group boundaries in oct_cells
    int64_t npairs = 0;
    DBuf<int32_t> pair_t, pair_tgt, pair_src, pair_goff;
    // level-adaptive trees only
    DBuf<int32_t> isleaf;           // [C]: 1 for a leaf
    DBuf<int32_t> flat;             // [C]: index in the tree's leaf table, -1 if not a leaf
    int32_t nleaf = 0, leaf0 = 0;   // leaves of this level: leaf table [leaf0, leaf0 + nleaf)
    DBuf<int32_t> x_off, x_leaf;    // X lists: CSR over the cells, leaf-table indices
    DBuf<int32_t> x_cells;          // cells whose X list is not empty
    int32_t nx_cells = 0;
};

}  // namespace bbfmm

struct bbfmm_tree {
    int64_t n = 0;
    int depth = 0;
    bbfmm_tree_params params{};
    float lo[3] = {0, 0, 0};
    float side = 1.f, scale = 1.f;
    int32_t max_leaf = 0;
    int64_t near_pairs = 0;
    bbfmm::DBuf<int32_t> perm;
    bbfmm::DBuf<float> xs, ys, zs;
    bbfmm::LevelData lv[bbfmm::kMaxLevels];
    bbfmm::DBuf<int32_t> nbr_off, nbr_idx;
    int64_t nbr_nnz = 0;
    bbfmm::DBuf<int32_t> tables;    // tvec[316][3], slot_t[8][189], t_slot[8][316]
    std::vector<int32_t> leaf_pb_h, leaf_pe_h;   // host copies of the leaf point ranges
    // Separate target and source sets: the points are [targets; sources]
    // (n_targets of them targets; 0 = one set, every point both).  Within a
    // leaf the targets come first (stable sort): targets [pb, te), sources
    // [sb, pe) with te == sb.
    int64_t n_targets = 0;
    bbfmm::DBuf<int32_t> leaf_sb, leaf_te;      // per leaf, only with separate sets
    std::vector<int32_t> leaf_te_h;             // host copy of the target ends (pe for one set)
    bbfmm_allocator hook{};         // allocator of the tree, inherited by its operators and plans
    // Level-adaptive tree: leaves on every level, gathered in one leaf table
    // (by level, then cell) on which the near field runs; nbr_off / nbr_idx
    // are then the U lists over that table.  W lists (per leaf) name cells
    // of any level >= 2; X lists live on the levels.
    bool adaptive = false;
    bbfmm::LevelData fleaf;         // C, keys, pb, pe of the leaf table
    bbfmm::DBuf<int32_t> fl_level, fl_cell;
    bbfmm::DBuf<int32_t> w_off, w_level, w_cell;
    int64_t w_nnz = 0;
    int leaf_level() const { return depth - 1; }
    // the leaves the near field and the leaf stages run over
    const bbfmm::LevelData &leaves() const { return adaptive ? fleaf : lv[depth - 1]; }
    const int32_t *src_begin() const { return n_targets ? leaf_sb.p : leaves().pb.p; }
    const int32_t *tgt_end() const { return n_targets ? leaf_te.p : leaves().pe.p; }
    int64_t n_out() const { return n_targets ? n_targets : n; }          // rows of phi
    int64_t n_in() const { return n - n_targets; }                       // rows of sigma
    double half_width(int level) const { return double(side) / double(1ull << (level + 1)); }
};

namespace bbfmm {

// Chebyshev constants in float, passed to kernels by value.
struct ChebConst {
    int n;
    float s[kMaxOrder];              // nodes cos((2m+1) pi / 2n)
    float w[kMaxOrder];              // 1 / prod_{k != m} (s_m - s_k)
    float T[2][kMaxOrder][kMaxOrder];// T[o][i][j] = l_i((2o-1)/2 + s_j/2)
};

// One compressed operator set (a level, or every level of a homogeneous kernel).
struct OpSet {
    int k = 0, kp = 0;               // rank and rank padded for MFMA tiles
    DBuf<double> U64, V64, C64;      // m x k, m x k, 316 x k x k
    DBuf<double> sv_fat, sv_thin;    // m each (empty when imported / eps = 0)
    DBuf<float> U32;                 // mp x kp: U, zero past (m, k)   (decompression)
    DBuf<float> VT32;                // kp x mp: V^T, zero past (k, m) (compression)
    DBuf<float> C32;                 // 316 x kp x kp (zero-padded), FP32 M2L
    DBuf<uint16_t> Chi, Clo;         // 316 x kp x kp bf16 halves, split-BF16 M2L
    DBuf<uint16_t> C16;              // 316 x kp x kp fp16 scaled by 2^e_t, FP16 M2L
    DBuf<float> Cinv;                // 316: 2^-e_t
    DBuf<float2> Ghat;               // FFT M2L: 316 x Q operator spectra (fft_m2l.hip)
};

struct PlanCache;
void plan_cache_destroy(PlanCache *c);

struct OpsLevel {
    OpSet *set = nullptr;
    double scale = 1.0;              // factor applied after M2L (h^m for homogeneous kernels)
};

}  // namespace bbfmm

struct bbfmm_ops {
    const bbfmm_tree *tree = nullptr;
    int n = 0, m = 0, mp = 0;        // order, n^3, n^3 padded to a multiple of 16
    int precision = 0;
    double eps = 0.0;
    int nodes = 0;                   // interpolation nodes: 0 Chebyshev, 1 equally spaced
    bbfmm::ChebConst cheb{};
    std::vector<std::unique_ptr<bbfmm::OpSet>> sets;
    bbfmm::OpsLevel lv[bbfmm::kMaxLevels];
    bbfmm_allocator hook{};          // allocator of the operators and of their plans
    // workspaces of bbfmm_matvec, kept per (r, stream) (see matvec.hip)
    std::mutex cache_mu;
    bbfmm::PlanCache *cache = nullptr;
    ~bbfmm_ops();
};

namespace bbfmm {

// --------------------------------------------------------------- entry ----
bbfmm_tree *build_tree_impl(const float *pts, int64_t n, const bbfmm_tree_params &p,
                            hipStream_t s);
// a tree over [targets; sources] (both device N x 3)
bbfmm_tree *build_tree_sets_impl(const float *targets, int64_t nt, const float *sources,
                                 int64_t ns, const bbfmm_tree_params &p, hipStream_t s);
bbfmm_ops *precompute_impl(const bbfmm_tree *t, double eps, int precision, hipStream_t s);
void precompute_check(double eps, int precision);   // argument checks, no device work
void cheb_setup(bbfmm_ops *ops, hipStream_t s);   // nodes of ops->nodes

// FFT M2L on equally spaced nodes (fft_m2l.hip): transform size P = 2n per
// axis, Q = (P/2 + 1) P^2 complex values per (cell, column)
int fft_size(int n);
int fft_freqs(int n);
void fft_operator_spectra(int kid, double a, int n, double h, const int32_t *tvec,
                          DBuf<float2> &Ghat, hipStream_t s);
void fft_forward(int n, const float *M, int mp, int64_t rows, float2 *Mhat, hipStream_t s);
void fft_inverse(int n, const float2 *Fhat, int64_t rows, float scale, bool accumulate, int mp,
                 float *F, hipStream_t s);
void fft_m2l(int n, const float2 *Mhat, const float2 *Ghat, const int32_t *itab,
             const uint64_t *keys, const int32_t *slot_t, int64_t cells, int r, float2 *Fhat,
             hipStream_t s);
// Spatial blocks of one level for the FFT M2L of a level-uniform tree: the
// level's cells in blocks of 4 x 4 x 4 (the cells whose keys agree above
// the lowest 6 bits); tgt[blk][key & 63] is the cell at that position or
// -1, halo[blk][(z * 8 + y) * 8 + x] the cell at block offset (x - 2, y - 2,
// z - 2) cells or -1.  Every interaction-list source of a block's targets
// lies in that 8 x 8 x 8 halo.
// slots[o * 189 + j] = t | base << 16: transfer vector t of slot j of
// octant o and the halo cell of that slot's source for the block's first
// parent (the others add 2 px + 16 py + 128 pz).
struct FftBlocks {
    DBuf<int32_t> tgt, halo, slots;
    int32_t nblk = 0;
};
void fft_build_blocks(const uint64_t *keys, int32_t C, int lvl, FftBlocks &b, hipStream_t s);
void fft_m2l_blocks(int n, const float2 *Mhat, const float2 *Ghat, const FftBlocks &b, int r,
                    float2 *Fhat, hipStream_t s);
void finalize_opset(OpSet &set, int m, int mp, int precision, hipStream_t s);

struct Plan;
// A plan's device memory comes from the thread's MemScope; its set-up work
// (launch lists, tile masks) is enqueued on `setup` and every product of
// the plan is ordered after it.  transient: no events and no side stream
// (for a plan that lives for one synchronous product).
Plan *plan_create_impl(const bbfmm_tree *t, const bbfmm_ops *o, int64_t r,
                       const bbfmm_plan_options *opt, hipStream_t setup, bool transient = false);
void plan_execute_impl(Plan *p, const float *sigma, float *phi, hipStream_t s);
int64_t plan_workspace_bytes(const Plan *p);
void plan_resolved_options(const Plan *p, bbfmm_plan_options *out);   // the choices in effect
void plan_destroy(Plan *p);
void plan_set_timing(Plan *p, bool on);
void plan_set_graph(Plan *p, bool on);
void plan_stage_times(Plan *p, double *ms, int64_t *execs, bool reset);
// bbfmm_matvec: a cached plan per (r, stream) of the operator set
void matvec_cached(bbfmm_ops *o, const float *sigma, int64_t r, float *phi, hipStream_t s);

// --------------------------------------------------------- primitives ----
// exclusive prefix sum of n int32 values (in may equal out); returns total
int64_t scan_exclusive(const int32_t *in, int32_t *out, int64_t n, hipStream_t s);
// stable LSD radix sort of (key, value) by the low `bits` bits of key
void radix_sort_pairs(uint64_t *keys, int32_t *vals, int64_t n, int bits, hipStream_t s);

}  // namespace bbfmm
