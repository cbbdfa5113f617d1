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

__global__ void k_iota_i32(int32_t *p, int64_t n) {
    int64_t i = int64_t(blockIdx.x) * kThreads + threadIdx.x;
    if (i < n) p[i] = int32_t(i);
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

// Sort key of a cell for the M2L tiles: its octant in the top 3 bits, then
// a 61-bit hash of which of its 189 interaction slots hold a source.  Cells
// of one octant with the same slot pattern (the interior, or one stretch of
// the boundary) get equal keys, so a stable sort keeps them together in
// Morton order and a tile's visited slots are those of all its targets.
__global__ void __launch_bounds__(kThreads)
k_tile_order_keys(const uint64_t *keys, const int32_t *itab, int32_t C, uint64_t *okey,
                  int32_t *idx) {
    const int32_t a = blockIdx.x * kThreads + threadIdx.x;
    if (a >= C) return;
    uint64_t h = 0xcbf29ce484222325ull;           // FNV-1a over the slot words
    const int32_t *row = itab + int64_t(a) * kSlots;
    for (int w = 0; w < (kSlots + 31) / 32; ++w) {
        uint32_t bits = 0;
        for (int b = 0; b < 32 && 32 * w + b < kSlots; ++b) bits |= uint32_t(row[32 * w + b] >= 0) << b;
        for (int k = 0; k < 4; ++k) {
            h ^= (bits >> (8 * k)) & 0xffu;
            h *= 0x100000001b3ull;
        }
    }
    okey[a] = (uint64_t(keys[a] & 7) << 61) | (h >> 3);
    idx[a] = a;
}

// ------------------------------------------- level-adaptive tree
// The adaptive tree (Section 2.1: split a cell only while it holds more than
// leaf_size points) is the uniform tree with the descendants of every such
// small cell removed.  Flags are computed top-down on the uniform tree's
// indices, then every level is compacted.

__global__ void __launch_bounds__(kThreads)
k_adapt_flags(const int32_t *pb, const int32_t *pe, const int32_t *parent, int32_t C, int finest,
              int leaf_size, const int32_t *keep_up, const int32_t *leaf_up, int32_t *keep,
              int32_t *leaf) {
    const int32_t c = blockIdx.x * kThreads + threadIdx.x;
    if (c >= C) return;
    int32_t k = 1;
    if (keep_up != nullptr) {
        const int32_t up = parent[c];
        k = (keep_up[up] && !leaf_up[up]) ? 1 : 0;
    }
    keep[c] = k;
    leaf[c] = (finest || pe[c] - pb[c] <= leaf_size) ? 1 : 0;
}

struct AdaptCompact {
    const uint64_t *keys;
    const int32_t *pb, *pe, *parent, *cb, *ce, *leaf, *keep, *pos;
    const int32_t *pos_up;      // new index of the level above (nullptr at the root)
    const int32_t *pos_down;    // new index of the level below (nullptr at the last level)
    int32_t C;
    uint64_t *okeys;
    int32_t *opb, *ope, *oparent, *ocb, *oce, *oleaf;
};

// A kept cell that is not a leaf keeps all of its children, which stay one
// contiguous run on the level below.
__global__ void __launch_bounds__(kThreads) k_adapt_compact(AdaptCompact a) {
    const int32_t c = blockIdx.x * kThreads + threadIdx.x;
    if (c >= a.C || !a.keep[c]) return;
    const int32_t j = a.pos[c];
    a.okeys[j] = a.keys[c];
    a.opb[j] = a.pb[c];
    a.ope[j] = a.pe[c];
    a.oparent[j] = a.pos_up != nullptr ? a.pos_up[a.parent[c]] : -1;
    const bool lf = a.leaf[c] != 0 || a.pos_down == nullptr;
    a.ocb[j] = lf ? -1 : a.pos_down[a.cb[c]];
    a.oce[j] = lf ? -1 : a.pos_down[a.ce[c] - 1] + 1;
    a.oleaf[j] = lf ? 1 : 0;
}

// leaf table entries of one level (rank = exclusive scan of the leaf flags)
__global__ void __launch_bounds__(kThreads)
k_adapt_table(const int32_t *leaf, const int32_t *rank, int32_t C, int lvl, int32_t off,
              const uint64_t *keys, const int32_t *pb, const int32_t *pe, int32_t *flat,
              uint64_t *fkey, int32_t *fpb, int32_t *fpe, int32_t *flev, int32_t *fcell) {
    const int32_t c = blockIdx.x * kThreads + threadIdx.x;
    if (c >= C) return;
    if (!leaf[c]) {
        flat[c] = -1;
        return;
    }
    const int32_t q = off + rank[c];
    flat[c] = q;
    fkey[q] = keys[c];
    fpb[q] = pb[c];
    fpe[q] = pe[c];
    flev[q] = lvl;
    fcell[q] = c;
}

// Per-level arrays of the adaptive tree, by value.
struct LevelTab {
    const uint64_t *keys[kMaxLevels];
    const int32_t *leaf[kMaxLevels], *flat[kMaxLevels], *cb[kMaxLevels], *ce[kMaxLevels];
    int32_t C[kMaxLevels];
    int32_t base[kMaxLevels + 1];   // global cell id = base[level] + cell
    int L;                          // last level
};

// Append buffers of the list construction.  A pass with null arrays only
// counts (n[0] U entries, n[1] frontier cells, n[2] W entries).
struct ListOut {
    unsigned long long *n;
    uint64_t *u;                    // (leaf << 32) | leaf-table index of the U leaf
    int32_t *fq, *flev, *fcell;     // frontier: (leaf, level, cell) adjacent, not a leaf
    uint64_t *w;                    // (leaf << 32) | global id of the W cell
};

__device__ inline void emit_u(const ListOut &o, int32_t q, int32_t v) {
    const unsigned long long i = atomicAdd(&o.n[0], 1ull);
    if (o.u) o.u[i] = (uint64_t(q) << 32) | uint32_t(v);
}
__device__ inline void emit_f(const ListOut &o, int32_t q, int lvl, int32_t c) {
    const unsigned long long i = atomicAdd(&o.n[1], 1ull);
    if (o.fq) { o.fq[i] = q; o.flev[i] = lvl; o.fcell[i] = c; }
}
__device__ inline void emit_w(const ListOut &o, int32_t q, int32_t g) {
    const unsigned long long i = atomicAdd(&o.n[2], 1ull);
    if (o.w) o.w[i] = (uint64_t(q) << 32) | uint32_t(g);
}

// closed boxes of two cells (level, Morton key) touch or overlap, measured
// in cells of the last level L
__device__ inline bool cells_adjacent(int la, uint64_t ka, int lb, uint64_t kb, int L) {
    const int32_t sa = 1 << (L - la), sb = 1 << (L - lb);
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const int32_t a0 = int32_t(compact3(ka >> d)) << (L - la);
        const int32_t b0 = int32_t(compact3(kb >> d)) << (L - lb);
        if (a0 > b0 + sb || b0 > a0 + sa) return false;
    }
    return true;
}

// Seeds, one thread per (leaf q, offset of its 3x3x3 neighbourhood on its
// own level): an existing same-level cell is a U leaf or a frontier cell
// (adjacent, to be opened); a missing one may lie inside a coarser leaf,
// which is then adjacent (U).
__global__ void __launch_bounds__(kThreads)
k_adapt_seed(LevelTab T, const uint64_t *fkey, const int32_t *flev, int32_t NL, ListOut o) {
    const int64_t g = int64_t(blockIdx.x) * kThreads + threadIdx.x;
    if (g >= int64_t(NL) * 27) return;
    const int32_t q = int32_t(g / 27);
    const int off = int(g % 27);
    const int lb = flev[q];
    const uint64_t key = fkey[q];
    const int x = int(compact3(key)) + off % 3 - 1;
    const int y = int(compact3(key >> 1)) + (off / 3) % 3 - 1;
    const int z = int(compact3(key >> 2)) + off / 9 - 1;
    const int lim = 1 << lb;
    if (x < 0 || y < 0 || z < 0 || x >= lim || y >= lim || z >= lim) return;
    const int32_t c = lookup(T.keys[lb], T.C[lb], morton3(x, y, z));
    if (c >= 0) {
        if (T.leaf[lb][c]) emit_u(o, q, T.flat[lb][c]);
        else emit_f(o, q, lb, c);
        return;
    }
    for (int l2 = lb - 1; l2 >= 0; --l2) {
        const int sh = lb - l2;
        const int32_t a = lookup(T.keys[l2], T.C[l2], morton3(x >> sh, y >> sh, z >> sh));
        if (a >= 0) {
            if (T.leaf[l2][a]) emit_u(o, q, T.flat[l2][a]);
            return;             // an existing non-leaf ancestor: the spot is empty
        }
    }
}

// One frontier step, one thread per (frontier cell, child slot): a child
// adjacent to the leaf is a U leaf or the next frontier; one that is not is
// a W cell (its parent, the frontier cell, is adjacent).
__global__ void __launch_bounds__(kThreads)
k_adapt_expand(LevelTab T, const uint64_t *fkey, const int32_t *flev, const int32_t *fq,
               const int32_t *fl, const int32_t *fc, int64_t nf, ListOut o) {
    const int64_t g = int64_t(blockIdx.x) * kThreads + threadIdx.x;
    if (g >= nf * 8) return;
    const int64_t e = g / 8;
    const int32_t q = fq[e];
    const int l = fl[e];
    const int32_t c = fc[e];
    const int32_t ch = T.cb[l][c] + int32_t(g % 8);
    if (ch >= T.ce[l][c]) return;
    const int lc = l + 1;
    if (cells_adjacent(lc, T.keys[lc][ch], flev[q], fkey[q], T.L)) {
        if (T.leaf[lc][ch]) emit_u(o, q, T.flat[lc][ch]);
        else emit_f(o, q, lc, ch);
    } else {
        emit_w(o, q, T.base[lc] + ch);
    }
}

// after a sort: flag[i] = 1 where entry i differs from entry i - 1
__global__ void __launch_bounds__(kThreads)
k_unique_flags(const uint64_t *v, int64_t n, int32_t *flag) {
    const int64_t i = int64_t(blockIdx.x) * kThreads + threadIdx.x;
    if (i < n) flag[i] = (i == 0 || v[i] != v[i - 1]) ? 1 : 0;
}

// sorted (row << 32 | value) entries -> CSR: counts per row and the values
__global__ void __launch_bounds__(kThreads)
k_csr_fill(const uint64_t *v, int64_t n, const int32_t *flag, const int32_t *pos, int32_t *cnt,
           int32_t *val) {
    const int64_t i = int64_t(blockIdx.x) * kThreads + threadIdx.x;
    if (i >= n || (flag != nullptr && !flag[i])) return;
    const int64_t j = flag != nullptr ? pos[i] : i;
    val[j] = int32_t(uint32_t(v[i]));
    atomicAdd(&cnt[int32_t(v[i] >> 32)], 1);
}

// global cell ids -> (level, cell)
__global__ void __launch_bounds__(kThreads)
k_split_gid(const int32_t *gid, int64_t n, LevelTab T, int32_t *lev, int32_t *cell) {
    const int64_t i = int64_t(blockIdx.x) * kThreads + threadIdx.x;
    if (i >= n) return;
    const int32_t v = gid[i];
    int l = 0;
    while (l < T.L && T.base[l + 1] <= v) ++l;
    lev[i] = l;
    cell[i] = v - T.base[l];
}

// W entry (leaf q, cell g) -> X entry (cell g, leaf q)
__global__ void __launch_bounds__(kThreads)
k_transpose_pairs(const uint64_t *w, int64_t n, uint64_t *x) {
    const int64_t i = int64_t(blockIdx.x) * kThreads + threadIdx.x;
    if (i < n) x[i] = (w[i] << 32) | (w[i] >> 32);
}

// per-level slice of a global CSR offset array, rebased to start at 0
__global__ void __launch_bounds__(kThreads)
k_rebase(const int32_t *goff, int32_t b, int32_t C, int32_t *off) {
    const int32_t c = blockIdx.x * kThreads + threadIdx.x;
    if (c <= C) off[c] = goff[b + c] - goff[b];
}

__global__ void __launch_bounds__(kThreads)
k_nonempty_flags(const int32_t *off, int32_t C, int32_t *flag) {
    const int32_t c = blockIdx.x * kThreads + threadIdx.x;
    if (c < C) flag[c] = off[c + 1] > off[c] ? 1 : 0;
}

__global__ void __launch_bounds__(kThreads)
k_compact_idx(const int32_t *flag, const int32_t *pos, int32_t C, int32_t *out) {
    const int32_t c = blockIdx.x * kThreads + threadIdx.x;
    if (c < C && flag[c]) out[pos[c]] = c;
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

// Compact every level to the cells of the level-adaptive tree, drop the
// trailing empty levels and gather the leaves of all levels into the leaf
// table (by level, then cell).
void adapt_levels(bbfmm_tree &t, int leaf_size, hipStream_t s) {
    const int D = t.depth, L = D - 1;
    std::vector<DBuf<int32_t>> keep(D), leaf(D), pos(D);
    std::vector<int32_t> newC(D);
    for (int l = 0; l < D; ++l) {
        const LevelData &lv = t.lv[l];
        keep[l].alloc(lv.C);
        leaf[l].alloc(lv.C);
        pos[l].alloc(lv.C);
        k_adapt_flags<<<grid(lv.C), kThreads, 0, s>>>(lv.pb.p, lv.pe.p, lv.parent.p, lv.C,
                                                      l == L ? 1 : 0, leaf_size,
                                                      l ? keep[l - 1].p : nullptr,
                                                      l ? leaf[l - 1].p : nullptr, keep[l].p,
                                                      leaf[l].p);
        BB_LAUNCH_CHECK();
        newC[l] = int32_t(scan_exclusive(keep[l].p, pos[l].p, lv.C, s));
    }
    int D2 = 0;
    while (D2 < D && newC[D2] > 0) ++D2;
    for (int l = 0; l < D2; ++l) {
        LevelData &lv = t.lv[l];
        const int32_t C2 = newC[l];
        DBuf<uint64_t> keys(C2);
        DBuf<int32_t> pb(C2), pe(C2), parent(C2), cb(C2), ce(C2), isleaf(C2);
        AdaptCompact a{};
        a.keys = lv.keys.p;
        a.pb = lv.pb.p;
        a.pe = lv.pe.p;
        a.parent = lv.parent.p;
        a.cb = lv.cb.p;
        a.ce = lv.ce.p;
        a.leaf = leaf[l].p;
        a.keep = keep[l].p;
        a.pos = pos[l].p;
        a.pos_up = l > 0 ? pos[l - 1].p : nullptr;
        a.pos_down = l + 1 < D2 ? pos[l + 1].p : nullptr;
        a.C = lv.C;
        a.okeys = keys.p;
        a.opb = pb.p;
        a.ope = pe.p;
        a.oparent = parent.p;
        a.ocb = cb.p;
        a.oce = ce.p;
        a.oleaf = isleaf.p;
        k_adapt_compact<<<grid(lv.C), kThreads, 0, s>>>(a);
        BB_LAUNCH_CHECK();
        BB_HIP(hipStreamSynchronize(s));
        lv.C = C2;
        lv.keys = std::move(keys);
        lv.pb = std::move(pb);
        lv.pe = std::move(pe);
        lv.parent = std::move(parent);
        lv.cb = std::move(cb);
        lv.ce = std::move(ce);
        lv.isleaf = std::move(isleaf);
    }
    for (int l = D2; l < D; ++l) t.lv[l] = LevelData();
    t.depth = D2;

    // the leaf table
    std::vector<DBuf<int32_t>> rank(D2);
    int32_t NL = 0;
    for (int l = 0; l < D2; ++l) {
        LevelData &lv = t.lv[l];
        rank[l].alloc(lv.C);
        lv.leaf0 = NL;
        lv.nleaf = int32_t(scan_exclusive(lv.isleaf.p, rank[l].p, lv.C, s));
        NL += lv.nleaf;
    }
    LevelData &F = t.fleaf;
    F.C = NL;
    F.keys.alloc(NL);
    F.pb.alloc(NL);
    F.pe.alloc(NL);
    t.fl_level.alloc(NL);
    t.fl_cell.alloc(NL);
    for (int l = 0; l < D2; ++l) {
        LevelData &lv = t.lv[l];
        lv.flat.alloc(lv.C);
        k_adapt_table<<<grid(lv.C), kThreads, 0, s>>>(lv.isleaf.p, rank[l].p, lv.C, l, lv.leaf0,
                                                      lv.keys.p, lv.pb.p, lv.pe.p, lv.flat.p,
                                                      F.keys.p, F.pb.p, F.pe.p, t.fl_level.p,
                                                      t.fl_cell.p);
        BB_LAUNCH_CHECK();
    }
    BB_HIP(hipStreamSynchronize(s));
}

// Sort (row << 32 | value) entries, optionally drop repeats, and write the
// CSR (off: rows + 1, val: the values).  Returns the entry count.
int64_t pairs_to_csr(DBuf<uint64_t> &v, int64_t n, int32_t rows, bool unique, DBuf<int32_t> &off,
                     DBuf<int32_t> &val, hipStream_t s) {
    int bits = 32;
    while (bits < 63 && (int64_t(1) << (bits - 32)) <= rows) ++bits;
    if (n > 0) {
        DBuf<int32_t> dummy(n);
        radix_sort_pairs(v.p, dummy.p, n, bits, s);
    }
    DBuf<int32_t> flag, pos;
    int64_t m = n;
    if (unique && n > 0) {
        flag.alloc(n);
        pos.alloc(n);
        k_unique_flags<<<grid(n), kThreads, 0, s>>>(v.p, n, flag.p);
        BB_LAUNCH_CHECK();
        m = scan_exclusive(flag.p, pos.p, n, s);
    }
    DBuf<int32_t> cnt(int64_t(rows) + 1);
    BB_HIP(hipMemsetAsync(cnt.p, 0, (size_t(rows) + 1) * sizeof(int32_t), s));
    val.alloc(m);
    if (n > 0) {
        k_csr_fill<<<grid(n), kThreads, 0, s>>>(v.p, n, flag.p, pos.p, cnt.p, val.p);
        BB_LAUNCH_CHECK();
    }
    off.alloc(int64_t(rows) + 1);
    scan_exclusive(cnt.p, off.p, int64_t(rows) + 1, s);
    BB_HIP(hipStreamSynchronize(s));
    return m;
}

// U, W and X lists of the level-adaptive tree (see k_adapt_seed and
// k_adapt_expand); also the near-field counts of the tree.
void adapt_lists(bbfmm_tree &t, hipStream_t s) {
    const int D = t.depth, L = D - 1;
    const int32_t NL = t.fleaf.C;
    LevelTab T{};
    T.L = L;
    T.base[0] = 0;
    for (int l = 0; l < D; ++l) {
        const LevelData &lv = t.lv[l];
        T.keys[l] = lv.keys.p;
        T.leaf[l] = lv.isleaf.p;
        T.flat[l] = lv.flat.p;
        T.cb[l] = lv.cb.p;
        T.ce[l] = lv.ce.p;
        T.C[l] = lv.C;
        T.base[l + 1] = T.base[l] + lv.C;
    }
    const int32_t ncells = T.base[D];
    DBuf<unsigned long long> cnt(3);
    unsigned long long hc[3];
    std::vector<DBuf<uint64_t>> uch, wch;
    std::vector<int64_t> un, wn;
    DBuf<int32_t> fq, fl, fc;
    int64_t nf = 0;
    // one list pass: count, allocate the appended chunks, fill
    auto pass = [&](auto launch) {
        BB_HIP(hipMemsetAsync(cnt.p, 0, sizeof(hc), s));
        ListOut o{cnt.p, nullptr, nullptr, nullptr, nullptr, nullptr};
        launch(o);
        BB_HIP(hipMemcpyAsync(hc, cnt.p, sizeof(hc), hipMemcpyDeviceToHost, s));
        BB_HIP(hipStreamSynchronize(s));
        DBuf<uint64_t> u(hc[0]), w(hc[2]);
        DBuf<int32_t> q2(hc[1]), l2(hc[1]), c2(hc[1]);
        BB_HIP(hipMemsetAsync(cnt.p, 0, sizeof(hc), s));
        o.u = u.p;
        o.fq = q2.p;
        o.flev = l2.p;
        o.fcell = c2.p;
        o.w = w.p;
        // a chunk the count found empty gets no buffer: its pointer stays null
        // and the fill pass writes nothing there
        launch(o);
        BB_HIP(hipStreamSynchronize(s));
        un.push_back(int64_t(hc[0]));
        wn.push_back(int64_t(hc[2]));
        uch.push_back(std::move(u));
        wch.push_back(std::move(w));
        fq = std::move(q2);
        fl = std::move(l2);
        fc = std::move(c2);
        nf = int64_t(hc[1]);
    };
    if (NL > 0)
        pass([&](const ListOut &o) {
            k_adapt_seed<<<unsigned(ceil_div(int64_t(NL) * 27, kThreads)), kThreads, 0, s>>>(
                T, t.fleaf.keys.p, t.fl_level.p, NL, o);
            BB_LAUNCH_CHECK();
        });
    for (int step = 0;; ++step) {       // `pass` updates nf, the frontier's size
        if (nf <= 0) break;
        BB_INTERNAL(step <= L, "adaptive list frontier did not drain");
        DBuf<int32_t> q0 = std::move(fq), l0 = std::move(fl), c0 = std::move(fc);
        const int64_t n0 = nf;
        pass([&](const ListOut &o) {
            k_adapt_expand<<<unsigned(ceil_div(n0 * 8, kThreads)), kThreads, 0, s>>>(
                T, t.fleaf.keys.p, t.fl_level.p, q0.p, l0.p, c0.p, n0, o);
            BB_LAUNCH_CHECK();
        });
    }
    auto gather = [&](std::vector<DBuf<uint64_t>> &ch, const std::vector<int64_t> &n,
                      DBuf<uint64_t> &all) {
        int64_t tot = 0;
        for (int64_t v : n) tot += v;
        all.alloc(tot);
        int64_t o = 0;
        for (size_t i = 0; i < ch.size(); ++i) {
            if (n[i] > 0)
                BB_HIP(hipMemcpyAsync(all.p + o, ch[i].p, n[i] * sizeof(uint64_t),
                                      hipMemcpyDeviceToDevice, s));
            o += n[i];
        }
        BB_HIP(hipStreamSynchronize(s));
        ch.clear();
        return tot;
    };
    DBuf<uint64_t> U, W;
    const int64_t nu = gather(uch, un, U);
    const int64_t nw = gather(wch, wn, W);
    t.nbr_nnz = pairs_to_csr(U, nu, NL, true, t.nbr_off, t.nbr_idx, s);

    // W: CSR over the leaf table, cells as (level, cell)
    DBuf<uint64_t> X(nw);
    if (nw > 0) {
        k_transpose_pairs<<<grid(nw), kThreads, 0, s>>>(W.p, nw, X.p);
        BB_LAUNCH_CHECK();
    }
    DBuf<int32_t> wg;
    t.w_nnz = pairs_to_csr(W, nw, NL, false, t.w_off, wg, s);
    t.w_level.alloc(t.w_nnz);
    t.w_cell.alloc(t.w_nnz);
    if (t.w_nnz > 0) {
        k_split_gid<<<grid(t.w_nnz), kThreads, 0, s>>>(wg.p, t.w_nnz, T, t.w_level.p, t.w_cell.p);
        BB_LAUNCH_CHECK();
    }
    // X: the transposed W pairs, CSR over all cells, then sliced per level
    DBuf<int32_t> xoff, xval;
    pairs_to_csr(X, nw, ncells, false, xoff, xval, s);
    std::vector<int32_t> hxoff(size_t(ncells) + 1);
    BB_HIP(hipMemcpyAsync(hxoff.data(), xoff.p, hxoff.size() * sizeof(int32_t),
                          hipMemcpyDeviceToHost, s));
    BB_HIP(hipStreamSynchronize(s));
    for (int l = 0; l < D; ++l) {
        LevelData &lv = t.lv[l];
        const int32_t b = T.base[l];
        lv.x_off.alloc(int64_t(lv.C) + 1);
        k_rebase<<<grid(int64_t(lv.C) + 1), kThreads, 0, s>>>(xoff.p, b, lv.C, lv.x_off.p);
        BB_LAUNCH_CHECK();
        const int32_t nx = hxoff[size_t(b) + lv.C] - hxoff[b];
        lv.x_leaf.alloc(nx);
        if (nx > 0)
            BB_HIP(hipMemcpyAsync(lv.x_leaf.p, xval.p + hxoff[b], nx * sizeof(int32_t),
                                  hipMemcpyDeviceToDevice, s));
        DBuf<int32_t> flag(lv.C), pos(lv.C);
        k_nonempty_flags<<<grid(lv.C), kThreads, 0, s>>>(lv.x_off.p, lv.C, flag.p);
        BB_LAUNCH_CHECK();
        lv.nx_cells = int32_t(scan_exclusive(flag.p, pos.p, lv.C, s));
        lv.x_cells.alloc(lv.nx_cells);
        if (lv.nx_cells > 0) {
            k_compact_idx<<<grid(lv.C), kThreads, 0, s>>>(flag.p, pos.p, lv.C, lv.x_cells.p);
            BB_LAUNCH_CHECK();
        }
        BB_HIP(hipStreamSynchronize(s));
    }

    // near-field sizes, from host copies of the leaf table and the U lists
    std::vector<int32_t> pb(NL), pe(NL), off(size_t(NL) + 1), idx(size_t(t.nbr_nnz));
    BB_HIP(hipMemcpyAsync(pb.data(), t.fleaf.pb.p, NL * sizeof(int32_t), hipMemcpyDeviceToHost, s));
    BB_HIP(hipMemcpyAsync(pe.data(), t.fleaf.pe.p, NL * sizeof(int32_t), hipMemcpyDeviceToHost, s));
    BB_HIP(hipMemcpyAsync(off.data(), t.nbr_off.p, off.size() * sizeof(int32_t),
                          hipMemcpyDeviceToHost, s));
    if (t.nbr_nnz > 0)
        BB_HIP(hipMemcpyAsync(idx.data(), t.nbr_idx.p, idx.size() * sizeof(int32_t),
                              hipMemcpyDeviceToHost, s));
    BB_HIP(hipStreamSynchronize(s));
    int64_t near = 0;
    int32_t most = 0;
    for (int32_t q = 0; q < NL; ++q) {
        int64_t src = 0;
        for (int32_t e = off[q]; e < off[q + 1]; ++e) src += pe[idx[e]] - pb[idx[e]];
        near += src * (pe[q] - pb[q]);
        most = std::max(most, pe[q] - pb[q]);
    }
    t.near_pairs = near;
    t.max_leaf = most;
}

void uniform_neighbors(bbfmm_tree &t, hipStream_t s);
void build_m2l_lists(bbfmm_tree &t, hipStream_t s);

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
    BB_REQUIRE(p.adaptive == 0 || p.adaptive == 1, "adaptive must be 0 or 1");
    if (p.adaptive) BB_REQUIRE(p.leaf_size >= 1, "leaf_size must be >= 1");
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

    if (p.adaptive) {
        t.adaptive = true;
        adapt_levels(t, p.leaf_size, s);
        adapt_lists(t, s);
    } else {
        uniform_neighbors(t, s);
    }
    build_m2l_lists(t, s);
    // host copies of the leaf point ranges, from which plans make their
    // near-field launch lists without reading the device
    const LevelData &leaves = t.leaves();
    t.leaf_pb_h.resize(size_t(leaves.C));
    t.leaf_pe_h.resize(size_t(leaves.C));
    BB_HIP(hipMemcpyAsync(t.leaf_pb_h.data(), leaves.pb.p, leaves.C * sizeof(int32_t),
                          hipMemcpyDeviceToHost, s));
    BB_HIP(hipMemcpyAsync(t.leaf_pe_h.data(), leaves.pe.p, leaves.C * sizeof(int32_t),
                          hipMemcpyDeviceToHost, s));
    BB_HIP(hipStreamSynchronize(s));
    t.leaf_te_h = t.leaf_pe_h;
    return tree.release();
}

namespace {

// Leaf neighbour lists N(.) of the uniform tree, and its leaf table (the
// leaf level).
void uniform_neighbors(bbfmm_tree &t, hipStream_t s) {
    const int L = t.leaf_level();
    const LevelData &leaf = t.lv[L];
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
    t.fl_level.alloc(leaf.C);
    t.fl_cell.alloc(leaf.C);
    k_fill_i32<<<grid(leaf.C), kThreads, 0, s>>>(t.fl_level.p, leaf.C, L);
    k_iota_i32<<<grid(leaf.C), kThreads, 0, s>>>(t.fl_cell.p, leaf.C);
    BB_LAUNCH_CHECK();
}

// Per level >= 2: the interaction table, the pairs grouped by transfer
// vector and the cells grouped by octant (Definition 2.1's I(.)).
void build_m2l_lists(bbfmm_tree &t, hipStream_t s) {
    const int L = t.leaf_level();
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
            DBuf<uint64_t> okey(C);
            k_tile_order_keys<<<grid(C), kThreads, 0, s>>>(lv.keys.p, lv.itab.p, lv.C, okey.p,
                                                           lv.oct_cells.p);
            BB_LAUNCH_CHECK();
            radix_sort_pairs(okey.p, lv.oct_cells.p, C, 64, s);
            k_group_offsets<<<1, 64, 0, s>>>(pos.p, lv.C, 8, lv.C, off.p);
            BB_LAUNCH_CHECK();
            BB_HIP(hipMemcpyAsync(lv.oct_off, off.p, 9 * sizeof(int32_t), hipMemcpyDeviceToHost, s));
            BB_HIP(hipStreamSynchronize(s));
        }
    }
}

}  // namespace

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
    BB_REQUIRE(p.adaptive == 0, "a level-adaptive tree takes one point set");
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
