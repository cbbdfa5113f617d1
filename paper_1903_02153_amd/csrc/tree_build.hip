// Octree construction on the GPU (Section 2.1, Definition 2.1).
//
//   bounding cube  -> float32 binning + 63-bit Morton key per point
//   (depth rule)   -> sort of the full keys, largest run per level
//   leaf sort      -> stable radix sort of the leaf key, permutation
//   cells          -> run heads + prefix sums, level by level up to the root
//   lists          -> leaf neighbour CSR; per level >= 2 the interaction
//                     table (cell x 189 slots) and the pair list grouped by
//                     transfer vector; cells grouped by octant for M2L tiles
//
// Everything is integer work after the binning, so the result is identical
// to any other implementation of the same definitions.  The binning is two
// correctly rounded float32 operations (__fsub_rn, __fmul_rn: no
// contraction into an FMA), which the FP64 oracle reproduces exactly.
#include "common.h"

namespace bbfmm {
namespace {

constexpr int kThreads = 256;

__device__ __host__ inline uint64_t spread3(uint32_t v) {
    uint64_t x = v & 0x1fffffu;
    x = (x | (x << 32)) & 0x1f00000000ffffull;
    x = (x | (x << 16)) & 0x1f0000ff0000ffull;
    x = (x | (x << 8)) & 0x100f00f00f00f00full;
    x = (x | (x << 4)) & 0x10c30c30c30c30c3ull;
    x = (x | (x << 2)) & 0x1249249249249249ull;
    return x;
}

__device__ inline uint32_t compact3(uint64_t x) {
    x &= 0x1249249249249249ull;
    x = (x ^ (x >> 2)) & 0x10c30c30c30c30c3ull;
    x = (x ^ (x >> 4)) & 0x100f00f00f00f00full;
    x = (x ^ (x >> 8)) & 0x1f0000ff0000ffull;
    x = (x ^ (x >> 16)) & 0x1f00000000ffffull;
    x = (x ^ (x >> 32)) & 0x1fffffull;
    return uint32_t(x);
}

__device__ inline uint64_t morton3(uint32_t x, uint32_t y, uint32_t z) {
    return spread3(x) | (spread3(y) << 1) | (spread3(z) << 2);
}

// index of key in sorted keys[0, n), or -1
__device__ inline int32_t lookup(const uint64_t *keys, int32_t n, uint64_t key) {
    int32_t lo = 0, hi = n;
    while (lo < hi) {
        int32_t mid = (lo + hi) >> 1;
        if (keys[mid] < key) lo = mid + 1; else hi = mid;
    }
    return (lo < n && keys[lo] == key) ? lo : -1;
}

__global__ void __launch_bounds__(kThreads)
k_bbox_partial(const float *pts, int64_t n, float *part, int32_t *bad) {
    __shared__ float smn[3][kThreads], smx[3][kThreads];
    float mn[3] = {INFINITY, INFINITY, INFINITY}, mx[3] = {-INFINITY, -INFINITY, -INFINITY};
    int nonfinite = 0;
    for (int64_t i = int64_t(blockIdx.x) * kThreads + threadIdx.x; i < n;
         i += int64_t(gridDim.x) * kThreads) {
        for (int d = 0; d < 3; ++d) {
            float v = pts[3 * i + d];
            if (!isfinite(v)) nonfinite = 1;
            mn[d] = fminf(mn[d], v);
            mx[d] = fmaxf(mx[d], v);
        }
    }
    if (nonfinite) atomicOr(bad, 1);
    for (int d = 0; d < 3; ++d) { smn[d][threadIdx.x] = mn[d]; smx[d][threadIdx.x] = mx[d]; }
    __syncthreads();
    for (int s = kThreads / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s)
            for (int d = 0; d < 3; ++d) {
                smn[d][threadIdx.x] = fminf(smn[d][threadIdx.x], smn[d][threadIdx.x + s]);
                smx[d][threadIdx.x] = fmaxf(smx[d][threadIdx.x], smx[d][threadIdx.x + s]);
            }
        __syncthreads();
    }
    if (threadIdx.x == 0)
        for (int d = 0; d < 3; ++d) {
            part[6 * blockIdx.x + d] = smn[d][0];
            part[6 * blockIdx.x + 3 + d] = smx[d][0];
        }
}

__global__ void __launch_bounds__(kThreads)
k_bbox_final(const float *part, int nparts, float *out) {
    __shared__ float s[6][kThreads];
    float v[6] = {INFINITY, INFINITY, INFINITY, -INFINITY, -INFINITY, -INFINITY};
    for (int i = threadIdx.x; i < nparts; i += kThreads)
        for (int d = 0; d < 3; ++d) {
            v[d] = fminf(v[d], part[6 * i + d]);
            v[3 + d] = fmaxf(v[3 + d], part[6 * i + 3 + d]);
        }
    for (int d = 0; d < 6; ++d) s[d][threadIdx.x] = v[d];
    __syncthreads();
    for (int st = kThreads / 2; st > 0; st >>= 1) {
        if (threadIdx.x < st)
            for (int d = 0; d < 3; ++d) {
                s[d][threadIdx.x] = fminf(s[d][threadIdx.x], s[d][threadIdx.x + st]);
                s[3 + d][threadIdx.x] = fmaxf(s[3 + d][threadIdx.x], s[3 + d][threadIdx.x + st]);
            }
        __syncthreads();
    }
    if (threadIdx.x < 6) out[threadIdx.x] = s[threadIdx.x][0];
}

// 63-bit Morton key of the 21-bit binned coordinates
__global__ void __launch_bounds__(kThreads)
k_quantize(const float *pts, int64_t n, float lox, float loy, float loz, float scale,
           uint64_t *key) {
#pragma clang fp contract(off)
    int64_t i = int64_t(blockIdx.x) * kThreads + threadIdx.x;
    if (i >= n) return;
    const float lo[3] = {lox, loy, loz};
    uint32_t q[3];
    for (int d = 0; d < 3; ++d) {
        float v = __fmul_rn(__fsub_rn(pts[3 * i + d], lo[d]), scale);
        float f = floorf(v);
        int64_t qi = f >= float(1 << kQBits) ? (1 << kQBits) - 1 : (f < 0.f ? 0 : int64_t(f));
        q[d] = uint32_t(qi);
    }
    key[i] = morton3(q[0], q[1], q[2]);
}

// largest number of points in one cell, for each level < nlev
__global__ void __launch_bounds__(kThreads)
k_level_maxcount(const uint64_t *keys, int64_t n, int nlev, int32_t *maxc) {
    int64_t i = int64_t(blockIdx.x) * kThreads + threadIdx.x;
    if (i >= n) return;
    for (int lvl = 0; lvl < nlev; ++lvl) {
        const int sh = 3 * (kQBits - lvl);
        const uint64_t pre = sh >= 64 ? 0 : keys[i] >> sh;
        if (i > 0 && (sh >= 64 ? 0 : keys[i - 1] >> sh) == pre) continue;
        int64_t lo = i + 1, hi = n;   // first index with a larger prefix
        while (lo < hi) {
            int64_t mid = (lo + hi) >> 1;
            uint64_t pm = sh >= 64 ? 0 : keys[mid] >> sh;
            if (pm <= pre) lo = mid + 1; else hi = mid;
        }
        atomicMax(&maxc[lvl], int32_t(lo - i));
    }
}

__global__ void __launch_bounds__(kThreads)
k_shift_keys(const uint64_t *in, int64_t n, int sh, uint64_t *out, int32_t *idx) {
    int64_t i = int64_t(blockIdx.x) * kThreads + threadIdx.x;
    if (i >= n) return;
    out[i] = in[i] >> sh;
    idx[i] = int32_t(i);
}

__global__ void __launch_bounds__(kThreads)
k_gather_points(const float *pts, const int32_t *perm, int64_t n, float *xs, float *ys,
                float *zs) {
    int64_t i = int64_t(blockIdx.x) * kThreads + threadIdx.x;
    if (i >= n) return;
    const int64_t j = perm[i];
    xs[i] = pts[3 * j];
    ys[i] = pts[3 * j + 1];
    zs[i] = pts[3 * j + 2];
}

// heads of runs of equal (key >> sh)
__global__ void __launch_bounds__(kThreads)
k_run_heads(const uint64_t *keys, int64_t n, int sh, int32_t *flag) {
    int64_t i = int64_t(blockIdx.x) * kThreads + threadIdx.x;
    if (i >= n) return;
    flag[i] = (i == 0 || (keys[i] >> sh) != (keys[i - 1] >> sh)) ? 1 : 0;
}

// cells of one level from the runs of the level below (or of the points)
__global__ void __launch_bounds__(kThreads)
k_run_fill(const uint64_t *keys, int64_t n, int sh, const int32_t *flag, const int32_t *pos,
           uint64_t *ckeys, int32_t *cbeg, int32_t *owner) {
    int64_t i = int64_t(blockIdx.x) * kThreads + threadIdx.x;
    if (i >= n) return;
    const int32_t c = pos[i] + flag[i] - 1;
    if (owner) owner[i] = c;
    if (flag[i]) {
        ckeys[c] = keys[i] >> sh;
        cbeg[c] = int32_t(i);
    }
}

__global__ void __launch_bounds__(kThreads)
k_run_end(const int32_t *cbeg, int32_t C, int32_t total, int32_t *cend) {
    int32_t c = blockIdx.x * kThreads + threadIdx.x;
    if (c >= C) return;
    cend[c] = (c + 1 < C) ? cbeg[c + 1] : total;
}

__global__ void __launch_bounds__(kThreads)
k_parent_ranges(const int32_t *cb, const int32_t *ce, int32_t C, const int32_t *child_pb,
                const int32_t *child_pe, int32_t *pb, int32_t *pe) {
    int32_t c = blockIdx.x * kThreads + threadIdx.x;
    if (c >= C) return;
    pb[c] = child_pb[cb[c]];
    pe[c] = child_pe[ce[c] - 1];
}

__global__ void k_fill_i32(int32_t *p, int64_t n, int32_t v) {
    int64_t i = int64_t(blockIdx.x) * kThreads + threadIdx.x;
    if (i < n) p[i] = v;
}

// leaf neighbour lists: pass 1 counts (idx == nullptr), pass 2 writes
__global__ void __launch_bounds__(kThreads)
k_neighbors(const uint64_t *keys, int32_t C, int L, const int32_t *off, int32_t *out,
            const int32_t *pb, const int32_t *pe, unsigned long long *near_pairs,
            int32_t *max_leaf) {
    int32_t a = blockIdx.x * kThreads + threadIdx.x;
    if (a >= C) return;
    const uint64_t key = keys[a];
    const int k[3] = {int(compact3(key)), int(compact3(key >> 1)), int(compact3(key >> 2))};
    const int lim = 1 << L;
    int32_t found[27];
    int nf = 0;
    for (int dz = -1; dz <= 1; ++dz)
        for (int dy = -1; dy <= 1; ++dy)
            for (int dx = -1; dx <= 1; ++dx) {
                int x = k[0] + dx, y = k[1] + dy, z = k[2] + dz;
                if (x < 0 || y < 0 || z < 0 || x >= lim || y >= lim || z >= lim) continue;
                int32_t b = lookup(keys, C, morton3(x, y, z));
                if (b >= 0) found[nf++] = b;
            }
    for (int i = 1; i < nf; ++i) {   // ascending cell index
        int32_t v = found[i];
        int j = i - 1;
        while (j >= 0 && found[j] > v) { found[j + 1] = found[j]; --j; }
        found[j + 1] = v;
    }
    if (off == nullptr) {
        out[a] = nf;
        unsigned long long src = 0;
        for (int i = 0; i < nf; ++i) src += unsigned(pe[found[i]] - pb[found[i]]);
        atomicAdd(near_pairs, src * unsigned(pe[a] - pb[a]));
        atomicMax(max_leaf, pe[a] - pb[a]);
    } else {
        for (int i = 0; i < nf; ++i) out[off[a] + i] = found[i];
    }
}

// interaction table: itab[a][j] = cell at k(a) + t(octant(a), j), or -1
__global__ void __launch_bounds__(kThreads)
k_itab(const uint64_t *keys, int32_t C, int lvl, const int32_t *tab, int32_t *itab) {
    int64_t g = int64_t(blockIdx.x) * kThreads + threadIdx.x;
    if (g >= int64_t(C) * kSlots) return;
    const int32_t a = int32_t(g / kSlots);
    const int j = int(g % kSlots);
    const uint64_t key = keys[a];
    const int o = int(key & 7);
    const int t = tab[3 * kNumT + o * kSlots + j];
    const int k[3] = {int(compact3(key)), int(compact3(key >> 1)), int(compact3(key >> 2))};
    const int lim = 1 << lvl;
    int x = k[0] + tab[3 * t], y = k[1] + tab[3 * t + 1], z = k[2] + tab[3 * t + 2];
    int32_t b = -1;
    if (x >= 0 && y >= 0 && z >= 0 && x < lim && y < lim && z < lim)
        b = lookup(keys, C, morton3(x, y, z));
    itab[g] = b;
}

// flags[t][a] = 1 when a has a source for transfer vector t
__global__ void __launch_bounds__(kThreads)
k_pair_flags(const uint64_t *keys, int32_t C, const int32_t *tab, const int32_t *itab,
             int32_t *flag) {
    int64_t g = int64_t(blockIdx.x) * kThreads + threadIdx.x;
    if (g >= int64_t(C) * kNumT) return;
    const int t = int(g / C);
    const int32_t a = int32_t(g % C);
    const int o = int(keys[a] & 7);
    const int j = tab[3 * kNumT + 8 * kSlots + o * kNumT + t];
    flag[g] = (j >= 0 && itab[int64_t(a) * kSlots + j] >= 0) ? 1 : 0;
}

__global__ void __launch_bounds__(kThreads)
k_pair_fill(const uint64_t *keys, int32_t C, const int32_t *tab, const int32_t *itab,
            const int32_t *flag, const int32_t *pos, int32_t *pt, int32_t *ptgt,
            int32_t *psrc) {
    int64_t g = int64_t(blockIdx.x) * kThreads + threadIdx.x;
    if (g >= int64_t(C) * kNumT || !flag[g]) return;
    const int t = int(g / C);
    const int32_t a = int32_t(g % C);
    const int o = int(keys[a] & 7);
    const int j = tab[3 * kNumT + 8 * kSlots + o * kNumT + t];
    const int32_t p = pos[g];
    pt[p] = t;
    ptgt[p] = a;
    psrc[p] = itab[int64_t(a) * kSlots + j];
}

// offsets of equal-stride groups: out[g] = pos[g * C] (g < G), out[G] = total
__global__ void k_group_offsets(const int32_t *pos, int32_t C, int G, int32_t total,
                                int32_t *out) {
    int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g > G) return;
    out[g] = g < G ? pos[int64_t(g) * C] : total;
}

__global__ void __launch_bounds__(kThreads)
k_octant_flags(const uint64_t *keys, int32_t C, int32_t *flag) {
    int64_t g = int64_t(blockIdx.x) * kThreads + threadIdx.x;
    if (g >= int64_t(C) * 8) return;
    const int o = int(g / C);
    flag[g] = int(keys[g % C] & 7) == o ? 1 : 0;
}

__global__ void __launch_bounds__(kThreads)
k_octant_fill(int32_t C, const int32_t *flag, const int32_t *pos, int32_t *cells) {
    int64_t g = int64_t(blockIdx.x) * kThreads + threadIdx.x;
    if (g >= int64_t(C) * 8 || !flag[g]) return;
    cells[pos[g]] = int32_t(g % C);
}

inline int grid(int64_t n) { return int(ceil_div(n, kThreads)); }

// Cells of a level from a sorted key array: runs of equal key >> sh.
// Returns the number of cells; fills keys/begin/end (end from `total`) and
// optionally the owning cell of every input element.
int32_t make_runs(const uint64_t *keys, int64_t n, int sh, int32_t total, LevelData &lv,
                  int32_t *owner, hipStream_t s) {
    DBuf<int32_t> flag(n), pos(n);
    k_run_heads<<<grid(n), kThreads, 0, s>>>(keys, n, sh, flag.p);
    BB_LAUNCH_CHECK();
    const int64_t C = scan_exclusive(flag.p, pos.p, n, s);
    lv.C = int32_t(C);
    lv.keys.alloc(C);
    DBuf<int32_t> beg(C), end(C);
    k_run_fill<<<grid(n), kThreads, 0, s>>>(keys, n, sh, flag.p, pos.p, lv.keys.p, beg.p, owner);
    BB_LAUNCH_CHECK();
    k_run_end<<<grid(C), kThreads, 0, s>>>(beg.p, int32_t(C), total, end.p);
    BB_LAUNCH_CHECK();
    BB_HIP(hipStreamSynchronize(s));
    lv.pb = std::move(beg);
    lv.pe = std::move(end);
    return int32_t(C);
}

}  // namespace

bbfmm_tree *build_tree_impl(const float *pts, int64_t n, const bbfmm_tree_params &p,
                            hipStream_t s) {
    BB_REQUIRE(pts != nullptr, "points is NULL");
    BB_REQUIRE(n >= 1 && n < (int64_t(1) << 31), "n must be in [1, 2^31)");
    BB_REQUIRE(p.cheb_order >= 2 && p.cheb_order <= kMaxOrder, "cheb_order must be in [2, 8]");
    BB_REQUIRE(p.kernel_id == BBFMM_K_INV_R || p.kernel_id == BBFMM_K_EXP ||
                   p.kernel_id == BBFMM_K_GAUSS || p.kernel_id == BBFMM_K_DIPOLE_X ||
                   p.kernel_id == BBFMM_K_POLY_TEST,
               "unknown kernel_id %d", p.kernel_id);
    BB_REQUIRE(p.kernel_id == BBFMM_K_INV_R || p.kernel_id == BBFMM_K_DIPOLE_X ||
                   (p.kernel_param > 0 && std::isfinite(p.kernel_param)),
               "kernel_param must be a positive finite length");
    BB_REQUIRE(p.fixed_depth >= 0 && p.fixed_depth <= kMaxLevels, "fixed_depth must be in [0, 22]");
    if (p.fixed_depth == 0) {
        BB_REQUIRE(p.leaf_size >= 1, "leaf_size must be >= 1");
        BB_REQUIRE(p.max_depth >= 1 && p.max_depth <= kMaxLevels, "max_depth must be in [1, 22]");
    }
    hipPointerAttribute_t attr{};
    BB_REQUIRE(hipPointerGetAttributes(&attr, pts) == hipSuccess &&
                   (attr.type == hipMemoryTypeDevice || attr.type == hipMemoryTypeManaged),
               "points must be a device pointer");

    std::unique_ptr<bbfmm_tree> tree(new bbfmm_tree());
    bbfmm_tree &t = *tree;
    t.n = n;
    t.params = p;

    // ---- bounding cube
    const int nparts = int(std::min<int64_t>(1024, ceil_div(n, kThreads)));
    DBuf<float> part(6 * nparts), box(6);
    DBuf<int32_t> bad(1);
    BB_HIP(hipMemsetAsync(bad.p, 0, sizeof(int32_t), s));
    k_bbox_partial<<<nparts, kThreads, 0, s>>>(pts, n, part.p, bad.p);
    BB_LAUNCH_CHECK();
    k_bbox_final<<<1, kThreads, 0, s>>>(part.p, nparts, box.p);
    BB_LAUNCH_CHECK();
    float hbox[6];
    int32_t hbad = 0;
    BB_HIP(hipMemcpyAsync(hbox, box.p, sizeof(hbox), hipMemcpyDeviceToHost, s));
    BB_HIP(hipMemcpyAsync(&hbad, bad.p, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    BB_HIP(hipStreamSynchronize(s));
    BB_REQUIRE(hbad == 0, "points contain a non-finite coordinate");
    float side = 0.f;
    for (int d = 0; d < 3; ++d) {
        t.lo[d] = hbox[d];
        volatile float ext = hbox[3 + d] - hbox[d];  // float32 subtraction
        side = std::max(side, float(ext));
    }
    if (!(side > 0.f)) side = 1.f;
    t.side = side;
    volatile float sc = float(1 << kQBits) / side;    // float32 division
    t.scale = sc;

    // ---- keys
    DBuf<uint64_t> key(n);
    k_quantize<<<grid(n), kThreads, 0, s>>>(pts, n, t.lo[0], t.lo[1], t.lo[2], t.scale, key.p);
    BB_LAUNCH_CHECK();

    int depth = p.fixed_depth;
    if (depth == 0) {
        DBuf<uint64_t> sk(n);
        DBuf<int32_t> dummy(n), maxc(p.max_depth);
        BB_HIP(hipMemcpyAsync(sk.p, key.p, n * sizeof(uint64_t), hipMemcpyDeviceToDevice, s));
        radix_sort_pairs(sk.p, dummy.p, n, 3 * kQBits, s);
        BB_HIP(hipMemsetAsync(maxc.p, 0, p.max_depth * sizeof(int32_t), s));
        k_level_maxcount<<<grid(n), kThreads, 0, s>>>(sk.p, n, p.max_depth, maxc.p);
        BB_LAUNCH_CHECK();
        std::vector<int32_t> hm(p.max_depth);
        BB_HIP(hipMemcpyAsync(hm.data(), maxc.p, p.max_depth * sizeof(int32_t),
                              hipMemcpyDeviceToHost, s));
        BB_HIP(hipStreamSynchronize(s));
        depth = p.max_depth;
        for (int d = 1; d <= p.max_depth; ++d)
            if (hm[d - 1] <= p.leaf_size) { depth = d; break; }
    }
    t.depth = depth;
    const int L = depth - 1;

    // ---- stable sort by leaf key
    DBuf<uint64_t> lkey(n);
    t.perm.alloc(n);
    k_shift_keys<<<grid(n), kThreads, 0, s>>>(key.p, n, 3 * (kQBits - L), lkey.p, t.perm.p);
    BB_LAUNCH_CHECK();
    key.release();
    radix_sort_pairs(lkey.p, t.perm.p, n, 3 * L, s);
    t.xs.alloc(n);
    t.ys.alloc(n);
    t.zs.alloc(n);
    k_gather_points<<<grid(n), kThreads, 0, s>>>(pts, t.perm.p, n, t.xs.p, t.ys.p, t.zs.p);
    BB_LAUNCH_CHECK();

    // ---- cells, leaf level then upwards
    LevelData &leaf = t.lv[L];
    make_runs(lkey.p, n, 0, int32_t(n), leaf, nullptr, s);
    lkey.release();
    leaf.cb.alloc(leaf.C);
    leaf.ce.alloc(leaf.C);
    k_fill_i32<<<grid(leaf.C), kThreads, 0, s>>>(leaf.cb.p, leaf.C, -1);
    k_fill_i32<<<grid(leaf.C), kThreads, 0, s>>>(leaf.ce.p, leaf.C, -1);
    BB_LAUNCH_CHECK();
    for (int lvl = L - 1; lvl >= 0; --lvl) {
        LevelData &ch = t.lv[lvl + 1], &pa = t.lv[lvl];
        ch.parent.alloc(ch.C);
        make_runs(ch.keys.p, ch.C, 3, ch.C, pa, ch.parent.p, s);
        // make_runs stored child ranges in pb/pe: they are cb/ce here
        pa.cb = std::move(pa.pb);
        pa.ce = std::move(pa.pe);
        pa.pb.alloc(pa.C);
        pa.pe.alloc(pa.C);
        k_parent_ranges<<<grid(pa.C), kThreads, 0, s>>>(pa.cb.p, pa.ce.p, pa.C, ch.pb.p, ch.pe.p,
                                                        pa.pb.p, pa.pe.p);
        BB_LAUNCH_CHECK();
    }
    t.lv[0].parent.alloc(t.lv[0].C);
    k_fill_i32<<<1, kThreads, 0, s>>>(t.lv[0].parent.p, t.lv[0].C, -1);
    BB_LAUNCH_CHECK();

    // ---- leaf neighbours
    DBuf<unsigned long long> npairs(1);
    DBuf<int32_t> maxleaf(1), cnt(leaf.C);
    BB_HIP(hipMemsetAsync(npairs.p, 0, sizeof(unsigned long long), s));
    BB_HIP(hipMemsetAsync(maxleaf.p, 0, sizeof(int32_t), s));
    k_neighbors<<<grid(leaf.C), kThreads, 0, s>>>(leaf.keys.p, leaf.C, L, nullptr, cnt.p,
                                                  leaf.pb.p, leaf.pe.p, npairs.p, maxleaf.p);
    BB_LAUNCH_CHECK();
    t.nbr_off.alloc(leaf.C + 1);
    t.nbr_nnz = scan_exclusive(cnt.p, t.nbr_off.p, leaf.C, s);
    {
        int32_t tot = int32_t(t.nbr_nnz);
        BB_HIP(hipMemcpyAsync(t.nbr_off.p + leaf.C, &tot, sizeof(int32_t), hipMemcpyHostToDevice, s));
        BB_HIP(hipStreamSynchronize(s));
    }
    t.nbr_idx.alloc(t.nbr_nnz);
    k_neighbors<<<grid(leaf.C), kThreads, 0, s>>>(leaf.keys.p, leaf.C, L, t.nbr_off.p,
                                                  t.nbr_idx.p, leaf.pb.p, leaf.pe.p, nullptr,
                                                  nullptr);
    BB_LAUNCH_CHECK();
    {
        unsigned long long hp = 0;
        BB_HIP(hipMemcpyAsync(&hp, npairs.p, sizeof(hp), hipMemcpyDeviceToHost, s));
        BB_HIP(hipMemcpyAsync(&t.max_leaf, maxleaf.p, sizeof(int32_t), hipMemcpyDeviceToHost, s));
        BB_HIP(hipStreamSynchronize(s));
        t.near_pairs = int64_t(hp);
    }

    // ---- M2L structures on levels >= 2
    const TransferTables &tt = transfer_tables();
    std::vector<int32_t> htab(3 * kNumT + 8 * kSlots + 8 * kNumT);
    for (int i = 0; i < kNumT; ++i)
        for (int d = 0; d < 3; ++d) htab[3 * i + d] = tt.tvec[i][d];
    for (int o = 0; o < 8; ++o) {
        for (int j = 0; j < kSlots; ++j) htab[3 * kNumT + o * kSlots + j] = tt.slot_t[o][j];
        for (int i = 0; i < kNumT; ++i) htab[3 * kNumT + 8 * kSlots + o * kNumT + i] = tt.t_slot[o][i];
    }
    t.tables.alloc(htab.size());
    DBuf<int32_t> &tab = t.tables;
    BB_HIP(hipMemcpyAsync(tab.p, htab.data(), htab.size() * sizeof(int32_t),
                          hipMemcpyHostToDevice, s));
    for (int lvl = 2; lvl <= L; ++lvl) {
        LevelData &lv = t.lv[lvl];
        const int64_t C = lv.C;
        lv.itab.alloc(C * kSlots);
        k_itab<<<grid(C * kSlots), kThreads, 0, s>>>(lv.keys.p, lv.C, lvl, tab.p, lv.itab.p);
        BB_LAUNCH_CHECK();
        {
            DBuf<int32_t> flag(C * kNumT), pos(C * kNumT);
            k_pair_flags<<<grid(C * kNumT), kThreads, 0, s>>>(lv.keys.p, lv.C, tab.p, lv.itab.p,
                                                              flag.p);
            BB_LAUNCH_CHECK();
            lv.npairs = scan_exclusive(flag.p, pos.p, C * kNumT, s);
            lv.pair_t.alloc(lv.npairs);
            lv.pair_tgt.alloc(lv.npairs);
            lv.pair_src.alloc(lv.npairs);
            lv.pair_goff.alloc(kNumT + 1);
            k_pair_fill<<<grid(C * kNumT), kThreads, 0, s>>>(lv.keys.p, lv.C, tab.p, lv.itab.p,
                                                             flag.p, pos.p, lv.pair_t.p,
                                                             lv.pair_tgt.p, lv.pair_src.p);
            BB_LAUNCH_CHECK();
            k_group_offsets<<<2, kThreads, 0, s>>>(pos.p, lv.C, kNumT, int32_t(lv.npairs),
                                                   lv.pair_goff.p);
            BB_LAUNCH_CHECK();
            BB_HIP(hipStreamSynchronize(s));
        }
        {
            DBuf<int32_t> flag(C * 8), pos(C * 8), off(9);
            k_octant_flags<<<grid(C * 8), kThreads, 0, s>>>(lv.keys.p, lv.C, flag.p);
            BB_LAUNCH_CHECK();
            const int64_t tot = scan_exclusive(flag.p, pos.p, C * 8, s);
            BB_INTERNAL(tot == C, "octant grouping lost cells");
            lv.oct_cells.alloc(C);
            k_octant_fill<<<grid(C * 8), kThreads, 0, s>>>(lv.C, flag.p, pos.p, lv.oct_cells.p);
            BB_LAUNCH_CHECK();
            k_group_offsets<<<1, 64, 0, s>>>(pos.p, lv.C, 8, lv.C, off.p);
            BB_LAUNCH_CHECK();
            BB_HIP(hipMemcpyAsync(lv.oct_off, off.p, 9 * sizeof(int32_t), hipMemcpyDeviceToHost, s));
            BB_HIP(hipStreamSynchronize(s));
        }
    }
    // host copies of the leaf point ranges, from which plans make their
    // near-field launch lists without reading the device
    t.leaf_pb_h.resize(size_t(leaf.C));
    t.leaf_pe_h.resize(size_t(leaf.C));
    BB_HIP(hipMemcpyAsync(t.leaf_pb_h.data(), leaf.pb.p, leaf.C * sizeof(int32_t),
                          hipMemcpyDeviceToHost, s));
    BB_HIP(hipMemcpyAsync(t.leaf_pe_h.data(), leaf.pe.p, leaf.C * sizeof(int32_t),
                          hipMemcpyDeviceToHost, s));
    BB_HIP(hipStreamSynchronize(s));
    t.leaf_te_h = t.leaf_pe_h;
    return tree.release();
}

// ------------------------------------------- separate target / source sets
namespace {

// te[a] = sb[a] = pb[a] + (number of targets in leaf a); the stable sort keeps
// the targets (indices < nt) ahead of the sources within a leaf, which
// `bad` records if it ever fails
__global__ void __launch_bounds__(kThreads)
k_split_leaves(const int32_t *pb, const int32_t *pe, const int32_t *perm, int nleaf, int32_t nt,
               int32_t *te, int32_t *sb, int32_t *bad) {
    const int a = blockIdx.x * kThreads + threadIdx.x;
    if (a >= nleaf) return;
    int i = pb[a];
    while (i < pe[a] && perm[i] < nt) ++i;
    te[a] = i;
    sb[a] = i;
    for (int j = i; j < pe[a]; ++j)
        if (perm[j] < nt) atomicOr(bad, 1);
}

}  // namespace

bbfmm_tree *build_tree_sets_impl(const float *targets, int64_t nt, const float *sources,
                                 int64_t ns, const bbfmm_tree_params &p, hipStream_t s) {
    BB_REQUIRE(targets != nullptr && sources != nullptr, "targets / sources is NULL");
    BB_REQUIRE(nt >= 1 && ns >= 1, "need at least one target and one source");
    BB_REQUIRE(nt + ns < (int64_t(1) << 31), "targets + sources must be < 2^31");
    std::unique_ptr<bbfmm_tree> tree;
    {
        DBuf<float> uni(size_t(nt + ns) * 3);
        BB_HIP(hipMemcpyAsync(uni.p, targets, size_t(nt) * 3 * sizeof(float),
                              hipMemcpyDeviceToDevice, s));
        BB_HIP(hipMemcpyAsync(uni.p + nt * 3, sources, size_t(ns) * 3 * sizeof(float),
                              hipMemcpyDeviceToDevice, s));
        tree.reset(build_tree_impl(uni.p, nt + ns, p, s));
        BB_HIP(hipStreamSynchronize(s));     // the union is read by the build only
    }
    bbfmm_tree &t = *tree;
    const LevelData &leaf = t.lv[t.leaf_level()];
    t.leaf_te.alloc(leaf.C);
    t.leaf_sb.alloc(leaf.C);
    DBuf<int32_t> bad(1);
    BB_HIP(hipMemsetAsync(bad.p, 0, sizeof(int32_t), s));
    k_split_leaves<<<grid(leaf.C), kThreads, 0, s>>>(leaf.pb.p, leaf.pe.p, t.perm.p, leaf.C,
                                                     int32_t(nt), t.leaf_te.p, t.leaf_sb.p, bad.p);
    BB_LAUNCH_CHECK();
    int32_t hbad = 0;
    t.leaf_te_h.resize(size_t(leaf.C));
    BB_HIP(hipMemcpyAsync(t.leaf_te_h.data(), t.leaf_te.p, leaf.C * sizeof(int32_t),
                          hipMemcpyDeviceToHost, s));
    BB_HIP(hipMemcpyAsync(&hbad, bad.p, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    BB_HIP(hipStreamSynchronize(s));
    BB_INTERNAL(hbad == 0, "targets do not lead their leaves");
    t.n_targets = nt;
    return tree.release();
}

}  // namespace bbfmm
