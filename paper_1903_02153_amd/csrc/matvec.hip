// The bbFMM matvec on the GPU (Section 2.3), FP32 throughout.
//
// Data in HBM (per level l >= 2; C_l cells, r right-hand sides, m = n^3,
// kp = compressed rank padded to 16):
//   M_l  [C_l][r][m]   multipole coefficients     (P2M / M2M)
//   Mh_l [C_l][r][kp]  compressed multipoles      V^T M
//   Fh_l [C_l][r][kp]  compressed locals          sum_t C_t Mh      (M2L)
//   F_l  [C_l][r][m]   local coefficients         scale U Fh + L2L
// Points stay sorted (structure of arrays) and sigma is gathered into that
// order once; phi is written straight back in the caller's order.
//
// Stages (one launch each, level-synchronous):
//   gather   sigma -> sorted order
//   p2m      per leaf: M = S^T sigma, then Mh = V^T M
//   m2m      per parent, levels L-1..2: M = sum_children T (x) T (x) T M_child,
//            three n x n mode products in LDS; then Mh = V^T M
//   m2l      per tile of same-octant targets: Fh += C_t Mh[source] for the
//            189 transfer vectors of that octant, fp32 MFMA 16x16x4
//   down     per cell, levels 2..L: F = scale U Fh + (T^T (x) T^T (x) T^T) F_parent
//   p2p      per 64 targets of a leaf: L2P of F plus the direct sum over
//            the neighbour leaves, staged through LDS
// No atomics on the data path: every output has one owner, so results are
// bitwise reproducible.
#include <type_traits>

#include "common.h"

namespace bbfmm {
namespace {

typedef float v4f __attribute__((ext_vector_type(4)));

constexpr int kThreads = 256;

// --------------------------------------------------------- geometry ----
__device__ inline uint32_t compact3(uint64_t x) {
    x &= 0x1249249249249249ull;
    x = (x ^ (x >> 2)) & 0x10c30c30c30c30c3ull;
    x = (x ^ (x >> 4)) & 0x100f00f00f00f00full;
    x = (x ^ (x >> 8)) & 0x1f0000ff0000ffull;
    x = (x ^ (x >> 16)) & 0x1f00000000ffffull;
    x = (x ^ (x >> 32)) & 0x1fffffull;
    return uint32_t(x);
}

// Cell centre lo + (2k+1) h as an unevaluated float pair hi + lo (exact
// product by FMA, exact sum by Knuth's two-sum), so that the local
// coordinate (x - c) / h keeps float precision at every depth.
__device__ inline void center_pair(float lo, uint32_t k, float h, float &chi, float &clo) {
#pragma clang fp contract(off)
    const float f = float(2u * k + 1u);
    const float p = __fmul_rn(f, h);
    const float e = __fmaf_rn(f, h, -p);
    const float s = __fadd_rn(lo, p);
    const float bb = __fsub_rn(s, lo);
    const float err = __fadd_rn(__fsub_rn(lo, __fsub_rn(s, bb)), __fsub_rn(p, bb));
    chi = s;
    clo = __fadd_rn(err, e);
}

__device__ inline float local_coord(float x, float chi, float clo, float inv_h) {
#pragma clang fp contract(off)
    return __fmul_rn(__fsub_rn(__fsub_rn(x, chi), clo), inv_h);
}

// l_m(xi) = w_m prod_{k != m} (xi - s_k)  for m < n
__device__ inline void lagrange(const ChebConst &cc, float xi, float *out) {
    const int n = cc.n;
    for (int m = 0; m < n; ++m) {
        float p = cc.w[m];
        for (int k = 0; k < n; ++k)
            if (k != m) p *= xi - cc.s[k];
        out[m] = p;
    }
}

// The same with the order fixed at compile time (loops unrolled, the node
// tables read with constant indices).
template <int N>
__device__ inline void lagrange_t(const ChebConst &cc, float xi, float *out) {
    float d[N];
#pragma unroll
    for (int k = 0; k < N; ++k) d[k] = xi - cc.s[k];
#pragma unroll
    for (int m = 0; m < N; ++m) {
        float p = cc.w[m];
#pragma unroll
        for (int k = 0; k < N; ++k)
            if (k != m) p *= d[k];
        out[m] = p;
    }
}

struct Geo {
    float lo[3];
    float h;        // half-width of a leaf
    float inv_h;
};

// ----------------------------------------------------------- kernels ----
// 1/r excludes coincident points (the kernel is singular there).  Instead of
// a compare and a select, r^2 is formed with a bias of -2^-126 folded into
// its first FMA: a zero distance gives a negative argument, v_rsq_f32
// returns NaN and the IEEE maximum with 0 returns 0.  For r^2 >= 2^-100 the
// bias is below half an ulp and r^2 is unchanged; pairs closer than about
// 1e-19 count as coincident.
constexpr float kInvRBias = 1.17549435e-38f;   // 2^-126

// Kernel values from coordinate differences that are already multiplied by
// the kernel's coordinate scale (coord_scale below), so that no per-pair
// multiply is left: exp(-r/a) = 2^-(r log2(e) / a) and exp(-r^2/a^2) =
// 2^-(r sqrt(log2 e) / a)^2 with the sign as a free source modifier.
template <int KID>
__device__ inline float kernel_eval(float dx, float dy, float dz) {
    if constexpr (KID == BBFMM_K_INV_R) {
        const float r2 = __fmaf_rn(dx, dx, __fmaf_rn(dy, dy, __fmaf_rn(dz, dz, -kInvRBias)));
        return __builtin_fmaxf(__frsqrt_rn(r2), 0.f);
    } else if constexpr (KID == BBFMM_K_EXP) {
        // v_sqrt_f32 and v_exp_f32 (1 ulp each)
        return __builtin_amdgcn_exp2f(-__builtin_amdgcn_sqrtf(dx * dx + dy * dy + dz * dz));
    } else if constexpr (KID == BBFMM_K_GAUSS) {
        return __builtin_amdgcn_exp2f(-(dx * dx + dy * dy + dz * dz));
    } else if constexpr (KID == BBFMM_K_DIPOLE_X) {
        // dx / r^3 with the same coincidence guard as 1/r (0 * 0 = 0)
        const float r2 = __fmaf_rn(dx, dx, __fmaf_rn(dy, dy, __fmaf_rn(dz, dz, -kInvRBias)));
        const float ir = __builtin_fmaxf(__frsqrt_rn(r2), 0.f);
        return dx * (ir * ir * ir);
    } else {
        const float u[3] = {dx, dy, dz};
        float p = 1.f;
        for (int d = 0; d < 3; ++d)
            p *= 1.f + u[d] * 0.5f - u[d] * u[d] * (1.f / 3.f) + u[d] * u[d] * u[d] * 0.2f;
        return p;
    }
}

// Factor applied to every coordinate before kernel_eval (1/r is scale-free
// up to a constant and is evaluated unscaled).
inline float coord_scale(int kid, double a) {
    const double log2e = 1.4426950408889634;
    switch (kid) {
    case BBFMM_K_INV_R: return 1.f;
    case BBFMM_K_DIPOLE_X: return 1.f;
    case BBFMM_K_EXP: return float(log2e / a);
    case BBFMM_K_GAUSS: return float(std::sqrt(log2e) / a);
    default: return float(1.0 / a);
    }
}

// ------------------------------------------------------------ gather ----
// sig_s[i][c] = sigma[perm[i] - base][c] for c < r, 0 for r <= c < ld and
// for points that are not sources (perm[i] < base: the targets of a tree
// over separate target and source sets, which come first)
__global__ void __launch_bounds__(kThreads)
k_gather_sigma(const float *sigma, const int32_t *perm, int64_t n, int r, int ld, int base,
               float *sig_s) {
    const int64_t g = int64_t(blockIdx.x) * kThreads + threadIdx.x;
    if (g >= n * ld) return;
    const int64_t i = g / ld;
    const int c = int(g % ld);
    const int u = perm[i] - base;
    sig_s[g] = (c < r && u >= 0) ? sigma[int64_t(u) * r + c] : 0.f;
}

// ----------------------------------------------------- up / down ----
// Node rows are padded from m = n^3 to mp (a multiple of 16) with zeros so
// that the compression GEMMs can read them with 16-byte loads.  The up /
// down interpolation kernels are compiled per order N, so node index
// arithmetic is by constants.

// P2M: M[leaf][c][node] = sum_p Lx_i1(p) Ly_i2(p) Lz_i3(p) sigma_p[c]   (grid:
// ceil(leaves / G) x r).  The wave holds G = 64 / n^2 leaves, one per group
// of n^2 lanes; lane (i2, i3) of a group keeps the n sums over i1 in
// registers and per point adds Ly Lz times the n values Lx sigma, which the
// whole group reads from one LDS row.  The points of all G leaves are
// requested together, so the wave waits for memory once per chunk.
template <int N>
__global__ void __launch_bounds__(64)
k_p2m(const float *xs, const float *ys, const float *zs, const int32_t *pb, const int32_t *pe,
      const uint64_t *keys, const int32_t *rows, int nleaf, Geo geo, ChebConst cc,
      const float *sig_s, int ld, int r, int mp, float *M) {
    constexpr int m = N * N * N, NP = N * N, G = 64 / NP;
    __shared__ float wx[G][64][N], wy[G][64][N], wz[G][64][N];   // Lx sigma, Ly, Lz per point
    const int lane = threadIdx.x;
    const int c = blockIdx.y;
    const int a0 = blockIdx.x * G;
    const int pq = lane % NP, g = lane / NP;
    const int i2 = pq % N, i3 = pq / N;
    // the leaf of every group (uniform loads)
    int lb[G], le[G];
    uint64_t key[G];
#pragma unroll
    for (int h = 0; h < G; ++h) {
        const bool ok = a0 + h < nleaf;
        lb[h] = ok ? pb[a0 + h] : 0;
        le[h] = ok ? pe[a0 + h] : 0;
        key[h] = ok ? keys[a0 + h] : 0;
    }
    int most = 0;
#pragma unroll
    for (int h = 0; h < G; ++h) most = max(most, le[h] - lb[h]);
    float acc[N];
#pragma unroll
    for (int k = 0; k < N; ++k) acc[k] = 0.f;
    for (int p0 = 0; p0 < most; p0 += 64) {
        float px[G], py[G], pz[G], ps[G];
#pragma unroll
        for (int h = 0; h < G; ++h) {                 // all loads first
            const int i = lb[h] + p0 + lane;
            const bool ok = i < le[h];
            const int q = ok ? i : lb[h];
            px[h] = xs[q];
            py[h] = ys[q];
            pz[h] = zs[q];
            ps[h] = ok ? sig_s[int64_t(q) * ld + c] : 0.f;
        }
        __syncthreads();                              // previous chunk consumed
#pragma unroll
        for (int h = 0; h < G; ++h) {
            if (lb[h] + p0 + lane >= le[h]) continue;
            float chi[3], clo[3], l[N];
            for (int d = 0; d < 3; ++d)
                center_pair(geo.lo[d], compact3(key[h] >> d), geo.h, chi[d], clo[d]);
            lagrange_t<N>(cc, local_coord(px[h], chi[0], clo[0], geo.inv_h), l);
#pragma unroll
            for (int k = 0; k < N; ++k) wx[h][lane][k] = l[k] * ps[h];
            lagrange_t<N>(cc, local_coord(py[h], chi[1], clo[1], geo.inv_h), l);
#pragma unroll
            for (int k = 0; k < N; ++k) wy[h][lane][k] = l[k];
            lagrange_t<N>(cc, local_coord(pz[h], chi[2], clo[2], geo.inv_h), l);
#pragma unroll
            for (int k = 0; k < N; ++k) wz[h][lane][k] = l[k];
        }
        __syncthreads();
        if (g < G) {
            int nmine = 0;
#pragma unroll
            for (int h = 0; h < G; ++h)
                if (h == g) nmine = min(64, le[h] - lb[h] - p0);
            for (int pp = 0; pp < nmine; ++pp) {
                const float t = wy[g][pp][i2] * wz[g][pp][i3];
#pragma unroll
                for (int k = 0; k < N; ++k) acc[k] = __fmaf_rn(wx[g][pp][k], t, acc[k]);
            }
        }
    }
    if (g < G && a0 + g < nleaf) {
        const int row = rows != nullptr ? rows[a0 + g] : a0 + g;
        float *out = M + (int64_t(row) * r + c) * mp;
#pragma unroll
        for (int k = 0; k < N; ++k) out[pq * N + k] = acc[k];
        for (int i = m + pq; i < mp; i += NP) out[i] = 0.f;
    }
}

// P2M for blocks of right-hand sides on FP32 MFMA: M[leaf][c][node] =
// sum_p S[p][node] sigma[p][c] as D = A B with A[node][p] = S[p][node]
// (lane node + 16 (p % 4) forms the Lagrange product itself from the
// points' 1D values in LDS) and B[p][c] = sigma (staged in LDS).  One
// workgroup per (leaf, 16 NCB columns); wave w owns the 16-node row blocks
// w, w + 4, ...  A column's arithmetic does not depend on the others.
template <int N, int NCB>
__global__ void __launch_bounds__(kThreads)
k_p2m_mfma(const float *xs, const float *ys, const float *zs, const int32_t *pb, const int32_t *pe,
           const uint64_t *keys, const int32_t *rows, Geo geo, ChebConst cc, const float *sig_s,
           int ld, int r, int mp, float *M) {
    constexpr int m = N * N * N;
    constexpr int NRBT = (m + 15) / 16;         // 16-node row blocks (mp = 16 NRBT)
    constexpr int RBQ = (NRBT + 3) / 4;         // row blocks per wave
    constexpr int CW = 16 * NCB;
    constexpr int SST = CW == 16 ? 16 : CW + 16;   // = 16 mod 32: rows k, k+1 on disjoint banks
    constexpr int PC = 64;                      // points per LDS chunk
    __shared__ float lv[PC][3][N];
    __shared__ __align__(16) float ss[PC * SST];
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int a = blockIdx.x, col0 = blockIdx.y * CW;
    const uint64_t key = keys[a];
    float chi[3], clo[3];
    for (int d = 0; d < 3; ++d) center_pair(geo.lo[d], compact3(key >> d), geo.h, chi[d], clo[d]);
    int n1[RBQ], n2[RBQ], n3[RBQ];
    float nw[RBQ];                              // 0 for the padding nodes m <= node < mp
#pragma unroll
    for (int q = 0; q < RBQ; ++q) {
        const int node = 16 * (wave + 4 * q) + (lane & 15);
        const int nd = node < m ? node : 0;
        nw[q] = node < m ? 1.f : 0.f;
        n1[q] = nd % N;
        n2[q] = (nd / N) % N;
        n3[q] = nd / (N * N);
    }
    v4f acc[RBQ][NCB];
#pragma unroll
    for (int q = 0; q < RBQ; ++q)
#pragma unroll
        for (int cb = 0; cb < NCB; ++cb) acc[q][cb] = v4f{0.f, 0.f, 0.f, 0.f};
    const int b = pb[a], e = pe[a];
    for (int p0 = b; p0 < e; p0 += PC) {
        const int np = min(PC, e - p0), npad = (np + 3) & ~3;
        __syncthreads();
        if (tid < PC) {
            if (tid < np) {
                const float p3[3] = {xs[p0 + tid], ys[p0 + tid], zs[p0 + tid]};
                for (int d = 0; d < 3; ++d) {
                    float l[kMaxOrder];
                    lagrange(cc, local_coord(p3[d], chi[d], clo[d], geo.inv_h), l);
#pragma unroll
                    for (int k = 0; k < N; ++k) lv[tid][d][k] = l[k];
                }
            } else {
#pragma unroll
                for (int d = 0; d < 3; ++d)
#pragma unroll
                    for (int k = 0; k < N; ++k) lv[tid][d][k] = 0.f;
            }
        }
        for (int g = tid; g < PC * (CW / 4); g += kThreads) {
            const int pe4 = g / (CW / 4), part = g % (CW / 4);
            float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
            if (pe4 < np) v = *reinterpret_cast<const float4 *>(sig_s + int64_t(p0 + pe4) * ld + col0 + 4 * part);
            *reinterpret_cast<float4 *>(&ss[pe4 * SST + 4 * part]) = v;
        }
        __syncthreads();
        for (int k0 = 0; k0 < npad; k0 += 4) {
            const int pp = k0 + (lane >> 4);
            float bv[NCB];
#pragma unroll
            for (int cb = 0; cb < NCB; ++cb) bv[cb] = ss[pp * SST + cb * 16 + (lane & 15)];
#pragma unroll
            for (int q = 0; q < RBQ; ++q) {
                if (wave + 4 * q >= NRBT) break;
                const float av = lv[pp][0][n1[q]] * lv[pp][1][n2[q]] * lv[pp][2][n3[q]] * nw[q];
#pragma unroll
                for (int cb = 0; cb < NCB; ++cb)
                    acc[q][cb] = __builtin_amdgcn_mfma_f32_16x16x4f32(av, bv[cb], acc[q][cb], 0, 0, 0);
            }
        }
    }
    // D[i][j] sits in lane j + 16 (i / 4), register i % 4: four consecutive nodes
    const int row = rows != nullptr ? rows[a] : a;
#pragma unroll
    for (int q = 0; q < RBQ; ++q) {
        if (wave + 4 * q >= NRBT) break;
        const int node0 = 16 * (wave + 4 * q) + 4 * (lane >> 4);
#pragma unroll
        for (int cb = 0; cb < NCB; ++cb) {
            const int c = col0 + cb * 16 + (lane & 15);
            if (c < r)
                *reinterpret_cast<float4 *>(M + (int64_t(row) * r + c) * mp + node0) =
                    make_float4(acc[q][cb][0], acc[q][cb][1], acc[q][cb][2], acc[q][cb][3]);
        }
    }
}

// ---------------------------------------------- M2M / L2L by pencils ----
// The translation between a cell and a child is the tensor product
// T_z (x) T_y (x) T_x of three n x n matrices (the 1D interpolation of the
// child's nodes, Section 2.3).  A group of n^2 lanes holds one n^3 block of
// one column as n^2 pencils of n values along one axis; a mode product along
// the pencil axis is n^2 register FMAs per lane with the matrix entries
// uniform across the wave (scalar operands), and two transposes through LDS
// turn the pencils to the next axes (z, then y, then x).  A wave takes
// G = 64 / n^2 columns of one parent.
template <int N>
struct Pencil {
    static constexpr int NP = N * N, G = 64 / NP, m = N * N * N;
};

// w[i] = sum_j T[o][i][j] v[j]  (trans: T[o][j][i])
template <int N, bool TRANS>
__device__ inline void mode1(const ChebConst &cc, int o, const float *v, float *w) {
#pragma unroll
    for (int i = 0; i < N; ++i) {
        float s = 0.f;
#pragma unroll
        for (int j = 0; j < N; ++j) s = __fmaf_rn(TRANS ? cc.T[o][j][i] : cc.T[o][i][j], v[j], s);
        w[i] = s;
    }
}

// One child translation of a block held as z-pencils (lane p = i1 + N i2
// holds i3 = 0..N-1); returns x-pencils (lane p = i2 + N i3 holds i1).
// buf: this group's N^3 floats of LDS.
template <int N, bool TRANS>
__device__ inline void translate3(const ChebConst &cc, int oct, const float *vz, float *buf,
                                  int p, bool on, float *out) {
    const int ox = oct & 1, oy = (oct >> 1) & 1, oz = (oct >> 2) & 1;
    float w[N], u[N];
#pragma unroll
    for (int k = 0; k < N; ++k) u[k] = 0.f;       // lanes outside the groups stay at 0
    mode1<N, TRANS>(cc, oz, vz, w);                 // along z
    if (on) {
#pragma unroll
        for (int k = 0; k < N; ++k) buf[p + N * N * k] = w[k];
    }
    __syncthreads();
    const int a1 = p % N, a3 = p / N;               // y-pencils: lane (i1, i3)
    if (on) {
#pragma unroll
        for (int k = 0; k < N; ++k) u[k] = buf[a1 + N * k + N * N * a3];
    }
    __syncthreads();
    mode1<N, TRANS>(cc, oy, u, w);                  // along y
    if (on) {
#pragma unroll
        for (int k = 0; k < N; ++k) buf[a1 + N * k + N * N * a3] = w[k];
    }
    __syncthreads();
    if (on) {                                       // x-pencils: lane (i2, i3)
#pragma unroll
        for (int k = 0; k < N; ++k) u[k] = buf[k + N * p];
    }
    __syncthreads();
    mode1<N, TRANS>(cc, ox, u, out);                // along x
}

// M2M: M[P][c] = sum over the children of (T (x) T (x) T) M[child][c]
// (grid: parents x column groups).  Every child's pencils are loaded before
// the first translation; children are summed in child order.  A cell
// without children (a leaf above the last level of an adaptive tree) is
// left to P2M.
template <int N>
__global__ void __launch_bounds__(64)
k_m2m_pen(const int32_t *cb, const int32_t *ce, const uint64_t *ckeys, const float *Mc,
          ChebConst cc, int r, int mp, float *M) {
    using PN = Pencil<N>;
    __shared__ float bufs[PN::G][PN::m];
    const int lane = threadIdx.x, g = lane / PN::NP, p = lane % PN::NP;
    const int P = blockIdx.x, c = blockIdx.y * PN::G + g;
    const bool on = g < PN::G && c < r;
    const int c0 = cb[P], nc = min(ce[P] - c0, 8);
    if (nc <= 0) return;
    float *buf = bufs[on ? g : 0];
    float v[8][N];
#pragma unroll
    for (int k = 0; k < 8; ++k)
#pragma unroll
        for (int j = 0; j < N; ++j)
            v[k][j] = (on && k < nc) ? Mc[(int64_t(c0 + k) * r + c) * mp + p + PN::NP * j] : 0.f;
    float acc[N];
#pragma unroll
    for (int j = 0; j < N; ++j) acc[j] = 0.f;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        if (k >= nc) break;
        float t[N];
        translate3<N, false>(cc, int(ckeys[c0 + k] & 7), v[k], buf, p, on, t);
#pragma unroll
        for (int j = 0; j < N; ++j) acc[j] += t[j];
    }
    if (on) {
        float *out = M + (int64_t(P) * r + c) * mp;
#pragma unroll
        for (int j = 0; j < N; ++j) out[j + N * p] = acc[j];
        for (int i = PN::m + p; i < mp; i += PN::NP) out[i] = 0.f;
    }
}

// L2L: F[child][c] = (T^T (x) T^T (x) T^T) F[P][c] for every child of P
// (grid: parents x column groups); the parent's pencils are loaded once.
template <int N>
__global__ void __launch_bounds__(64)
k_l2l_pen(const int32_t *cb, const int32_t *ce, const uint64_t *ckeys, const float *Fp,
          ChebConst cc, int r, int mp, float *F) {
    using PN = Pencil<N>;
    __shared__ float bufs[PN::G][PN::m];
    const int lane = threadIdx.x, g = lane / PN::NP, p = lane % PN::NP;
    const int P = blockIdx.x, c = blockIdx.y * PN::G + g;
    const bool on = g < PN::G && c < r;
    const int c0 = cb[P], nc = min(ce[P] - c0, 8);
    if (nc <= 0) return;
    float *buf = bufs[on ? g : 0];
    float v[N];
#pragma unroll
    for (int j = 0; j < N; ++j) v[j] = on ? Fp[(int64_t(P) * r + c) * mp + p + PN::NP * j] : 0.f;
    for (int k = 0; k < nc; ++k) {
        float t[N];
        translate3<N, true>(cc, int(ckeys[c0 + k] & 7), v, buf, p, on, t);
        if (on) {
            float *out = F + (int64_t(c0 + k) * r + c) * mp;
#pragma unroll
            for (int j = 0; j < N; ++j) out[j + N * p] = t[j];
            for (int i = PN::m + p; i < mp; i += PN::NP) out[i] = 0.f;
        }
    }
}

// Y[R][N] = alpha X[R][K] Bt[N][K]^T + beta Y with FP32 MFMA 16x16x4, where
// X is the sum of nsum arrays xstride floats apart (the partial F^ of a
// split M2L); K a
// multiple of 16 and both operands zero beyond the true K.  A wave owns 16
// rows x 64 columns; operands are read straight from global memory with
// 16-byte loads along K (same permuted-K trick as the M2L kernel).
// Compression: Mh = M VT^T;  decompression: F = scale Fh U^T (+ F).
// Output formats of the compression GEMM (the operand format of the M2L).
enum { kOutF32 = 0, kOutBF16X3 = 1, kOutF16S = 2 };

__device__ inline uint16_t to_bf16(float x) { return __builtin_bit_cast(uint16_t, static_cast<__bf16>(x)); }
__device__ inline float from_bf16(uint16_t b) { return static_cast<float>(__builtin_bit_cast(__bf16, b)); }
__device__ inline uint16_t to_f16(float x) { return __builtin_bit_cast(uint16_t, static_cast<_Float16>(x)); }

template <int OUT>
__global__ void __launch_bounds__(kThreads)
k_gemm_nt(const float *X, int64_t ldx, int nsum, int64_t xstride, const float *Bt, int64_t ldb,
          float *Y, int64_t ldy, int64_t R, int Ncol, int K, float alpha, float beta,
          uint16_t *Yh, uint16_t *Yl, float *Sinv, int nchunk) {
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int64_t row0 = int64_t(blockIdx.x) * 64 + wave * 16;
    const int col0 = blockIdx.y * 64;
    const int64_t arow = row0 + (lane & 15);
    const float *xa = X + arow * ldx + 4 * (lane >> 4);
    const float *bb[4];
    bool bok[4];
#pragma unroll
    for (int cb = 0; cb < 4; ++cb) {
        const int bc = col0 + cb * 16 + (lane & 15);
        bok[cb] = bc < Ncol;
        bb[cb] = Bt + int64_t(bok[cb] ? bc : 0) * ldb + 4 * (lane >> 4);
    }
    const bool aok = arow < R;
    v4f acc[4];
    for (int cb = 0; cb < 4; ++cb) acc[cb] = v4f{0.f, 0.f, 0.f, 0.f};
    for (int k0 = 0; k0 < K; k0 += 16) {
        float4 a4 = make_float4(0.f, 0.f, 0.f, 0.f);
        if (aok)
            for (int q = 0; q < nsum; ++q) {   // fixed order: reproducible
                const float4 v = *reinterpret_cast<const float4 *>(xa + q * xstride + k0);
                a4.x += v.x; a4.y += v.y; a4.z += v.z; a4.w += v.w;
            }
        float4 b4[4];
#pragma unroll
        for (int cb = 0; cb < 4; ++cb)
            b4[cb] = bok[cb] ? *reinterpret_cast<const float4 *>(bb[cb] + k0) : make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
        for (int cb = 0; cb < 4; ++cb) acc[cb] = __builtin_amdgcn_mfma_f32_16x16x4f32(a4.x, b4[cb].x, acc[cb], 0, 0, 0);
#pragma unroll
        for (int cb = 0; cb < 4; ++cb) acc[cb] = __builtin_amdgcn_mfma_f32_16x16x4f32(a4.y, b4[cb].y, acc[cb], 0, 0, 0);
#pragma unroll
        for (int cb = 0; cb < 4; ++cb) acc[cb] = __builtin_amdgcn_mfma_f32_16x16x4f32(a4.z, b4[cb].z, acc[cb], 0, 0, 0);
#pragma unroll
        for (int cb = 0; cb < 4; ++cb) acc[cb] = __builtin_amdgcn_mfma_f32_16x16x4f32(a4.w, b4[cb].w, acc[cb], 0, 0, 0);
    }
    if constexpr (OUT == kOutF32) {
        // through LDS, so that each row of the wave's 16 x 64 tile is read
        // (beta) and written as 256 contiguous bytes
        __shared__ float tile[4][16][64 + 4];
#pragma unroll
        for (int cb = 0; cb < 4; ++cb)
#pragma unroll
            for (int v = 0; v < 4; ++v) tile[wave][4 * (lane >> 4) + v][cb * 16 + (lane & 15)] = acc[cb][v];
        __syncthreads();
#pragma unroll
        for (int it = 0; it < 4; ++it) {
            const int idx = it * 64 + lane, rr = idx >> 4, q = idx & 15;
            const int64_t row = row0 + rr;
            const int col = col0 + 4 * q;
            if (row >= R || col >= Ncol) continue;
            const float4 d = *reinterpret_cast<const float4 *>(&tile[wave][rr][4 * q]);
            float4 *y = reinterpret_cast<float4 *>(Y + row * ldy + col);
            float4 o = make_float4(alpha * d.x, alpha * d.y, alpha * d.z, alpha * d.w);
            if (beta != 0.f) {
                const float4 old = *y;
                o = make_float4(o.x + beta * old.x, o.y + beta * old.y, o.z + beta * old.z, o.w + beta * old.w);
            }
            *y = o;
        }
    } else {
        // 16-bit outputs, converted in registers and written through LDS so
        // that each row of the wave's 16 x 64 tile leaves as 128 contiguous
        // bytes per plane.  BF16x3: x = hi + lo with hi = bf16(x), lo =
        // bf16(x - hi).  Scaled FP16: one power-of-two scale per (row,
        // 64-column chunk), max |x| 2^e in [2^14, 2^15).
        constexpr int NPL = OUT == kOutBF16X3 ? 2 : 1;
        __shared__ uint16_t tile16[NPL][4][16][64 + 8];
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int rr = 4 * (lane >> 4) + v;
            if constexpr (OUT == kOutBF16X3) {
#pragma unroll
                for (int cb = 0; cb < 4; ++cb) {
                    const float x = alpha * acc[cb][v];
                    const uint16_t h = to_bf16(x);
                    tile16[0][wave][rr][cb * 16 + (lane & 15)] = h;
                    tile16[NPL - 1][wave][rr][cb * 16 + (lane & 15)] = to_bf16(x - from_bf16(h));
                }
            } else {
                float mx = 0.f;
#pragma unroll
                for (int cb = 0; cb < 4; ++cb) mx = fmaxf(mx, bok[cb] ? fabsf(alpha * acc[cb][v]) : 0.f);
                for (int msk = 1; msk < 16; msk <<= 1) mx = fmaxf(mx, __shfl_xor(mx, msk, 64));
                const int e = mx > 0.f ? max(-126, min(126, 14 - ilogbf(mx))) : 0;
#pragma unroll
                for (int cb = 0; cb < 4; ++cb)
                    tile16[0][wave][rr][cb * 16 + (lane & 15)] = to_f16(ldexpf(alpha * acc[cb][v], e));
                const int64_t row = row0 + rr;
                if (row < R && (lane & 15) == 0) Sinv[row * nchunk + blockIdx.y] = ldexpf(1.f, -e);
            }
        }
        __syncthreads();
        // 16 rows x 8 pieces of 8 halves per plane: two pieces per lane
#pragma unroll
        for (int it = 0; it < 2; ++it) {
            const int idx = it * 64 + lane, rr = idx >> 3, q = idx & 7;
            const int64_t row = row0 + rr;
            const int col = col0 + 8 * q;
            if (row >= R || col >= Ncol) continue;
#pragma unroll
            for (int pl = 0; pl < NPL; ++pl) {
                uint16_t *dst = (pl == 0 ? Yh : Yl) + row * ldy + col;
                *reinterpret_cast<uint4 *>(dst) = *reinterpret_cast<const uint4 *>(&tile16[pl][wave][rr][8 * q]);
            }
        }
    }
}

// ------------------------------------------- fused leaf upward pass ----
// P2M, compression and M2M of the leaf level in one kernel (Section 2.3,
// upward pass; Section 2.5: the right-hand sides as the columns of matrix
// products).  A workgroup takes one parent cell and 16 right-hand sides.
// For each child leaf in turn it
//   A. forms M = S^T sigma (n^3 x 16) on FP32 MFMA into LDS (as k_p2m_mfma:
//      wave w owns the 16-node row blocks w, w + 4, ...);
//   B. compresses it, M^ = V^T M (kp x 16) on FP32 MFMA with V^T read from
//      global memory (wave w owns the rank row blocks w, w + 4, ...), and
//      writes M^ in the M2L operand format (as k_gemm_nt's epilogues);
//   C. adds its translation to the parent's coefficients, held as pencils
//      in registers (as k_m2m_pen; a thread owns up to four (column,
//      pencil) pairs).
// The leaves' full coefficients never reach HBM; the parent's are written
// once.  Per output the sums run in the same order as in the separate
// kernels except that M feeds the compression from LDS.
struct LeafUpArgs {
    const float *xs, *ys, *zs;
    const int32_t *sb, *pe;          // leaf source ranges (tree order)
    const uint64_t *keys;            // leaf keys
    const int32_t *pcb, *pce;        // children of each parent (level L-1)
    const float *sig_s;
    int ld, r, mp, kp, nchunk;
    const float *VT;                 // kp x mp: V^T of the leaf level
    float *Mh;                       // FP32 operands [leaf][r][kp]
    uint16_t *Mh16, *Ml16;           // 16-bit operands [leaf][r][kp]
    float *Msinv;                    // fp16: inverse scales [leaf][r][nchunk]
    float *Mpar;                     // parent coefficients [parent][r][mp]
};

template <int N, int OUT>
__global__ void __launch_bounds__(kThreads)
k_leaf_up(LeafUpArgs a, Geo geo, ChebConst cc) {
    constexpr int m = N * N * N, NP = N * N;
    constexpr int MPAD = ((m + 15) / 16) * 16;    // == mp
    constexpr int NRBT = MPAD / 16;               // node row blocks
    constexpr int RBQ = (NRBT + 3) / 4;           // ... per wave
    constexpr int MS = 17;                        // LDS row stride of M (16 columns + pad)
    constexpr int PC = 64;                        // points per staging chunk
    constexpr int TPT = (16 * NP + kThreads - 1) / kThreads;   // pencils per thread
    constexpr int STAGE = PC * 3 * N + PC * 16;   // floats: Lagrange values + sigma
    constexpr int SCR = 16 * m;                   // floats: pencil transposes
    __shared__ float Ms[MPAD * MS];
    __shared__ float pool[STAGE > SCR ? STAGE : SCR];
    __shared__ float cmax[4][16];
    float (*lv)[3][N] = reinterpret_cast<float (*)[3][N]>(pool);
    float *ss = pool + PC * 3 * N;                // [PC][16]
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int P = blockIdx.x, col0 = blockIdx.y * 16;
    const int c0 = a.pcb[P], nc = a.pce[P] - c0;
    const int r = a.r, kp = a.kp, nrb = kp / 16;
    // node decomposition of this lane's P2M rows
    int n1[RBQ], n2[RBQ], n3[RBQ];
    float nw[RBQ];
#pragma unroll
    for (int q = 0; q < RBQ; ++q) {
        const int node = 16 * (wave + 4 * q) + (lane & 15);
        const int nd = node < m ? node : 0;
        nw[q] = node < m ? 1.f : 0.f;
        n1[q] = nd % N;
        n2[q] = (nd / N) % N;
        n3[q] = nd / NP;
    }
    float par[TPT][N];
#pragma unroll
    for (int u = 0; u < TPT; ++u)
#pragma unroll
        for (int k = 0; k < N; ++k) par[u][k] = 0.f;

    for (int ci = 0; ci < nc; ++ci) {
        const int c = c0 + ci;
        const uint64_t key = a.keys[c];
        // ---- A: P2M into Ms
        float chi[3], clo[3];
        for (int d = 0; d < 3; ++d) center_pair(geo.lo[d], compact3(key >> d), geo.h, chi[d], clo[d]);
        v4f acc[RBQ];
#pragma unroll
        for (int q = 0; q < RBQ; ++q) acc[q] = v4f{0.f, 0.f, 0.f, 0.f};
        const int b = a.sb[c], e = a.pe[c];
        for (int p0 = b; p0 < e; p0 += PC) {
            const int np = min(PC, e - p0), npad = (np + 3) & ~3;
            __syncthreads();                      // previous chunk (or Ms / pool users) done
            if (tid < PC) {
                if (tid < np) {
                    const float p3[3] = {a.xs[p0 + tid], a.ys[p0 + tid], a.zs[p0 + tid]};
                    for (int d = 0; d < 3; ++d) {
                        float l[kMaxOrder];
                        lagrange(cc, local_coord(p3[d], chi[d], clo[d], geo.inv_h), l);
#pragma unroll
                        for (int k = 0; k < N; ++k) lv[tid][d][k] = l[k];
                    }
                } else {
#pragma unroll
                    for (int d = 0; d < 3; ++d)
#pragma unroll
                        for (int k = 0; k < N; ++k) lv[tid][d][k] = 0.f;
                }
            }
            for (int g = tid; g < PC * 16; g += kThreads) {
                const int pp = g / 16, j = g % 16;
                ss[g] = (pp < np && col0 + j < r) ? a.sig_s[int64_t(p0 + pp) * a.ld + col0 + j] : 0.f;
            }
            __syncthreads();
            for (int k0 = 0; k0 < npad; k0 += 4) {
                const int pp = k0 + (lane >> 4);
                const float bv = ss[pp * 16 + (lane & 15)];
#pragma unroll
                for (int q = 0; q < RBQ; ++q) {
                    if (wave + 4 * q >= NRBT) break;
                    const float av = lv[pp][0][n1[q]] * lv[pp][1][n2[q]] * lv[pp][2][n3[q]] * nw[q];
                    acc[q] = __builtin_amdgcn_mfma_f32_16x16x4f32(av, bv, acc[q], 0, 0, 0);
                }
            }
        }
        __syncthreads();                          // pool free; Ms readers of the last child done
        // D[i][j] in lane j + 16 (i / 4), register i % 4
#pragma unroll
        for (int q = 0; q < RBQ; ++q) {
            if (wave + 4 * q >= NRBT) break;
            const int node0 = 16 * (wave + 4 * q) + 4 * (lane >> 4);
#pragma unroll
            for (int v = 0; v < 4; ++v) Ms[(node0 + v) * MS + (lane & 15)] = acc[q][v];
        }
        __syncthreads();
        // ---- B: compression V^T M from Ms.  D[i = rank][j = column] of a
        // row block sits in lane j + 16 (i / 4), register i % 4.
        // (the operator rows of GB 16-node steps are requested together; two
        // accumulators interleave the dependent MFMA chain)
        auto compress_block = [&](int rb) -> v4f {
            constexpr int NK = MPAD / 16, GB = 4;
            v4f d0 = v4f{0.f, 0.f, 0.f, 0.f}, d1 = d0;
            const float *vrow = a.VT + int64_t(rb * 16 + (lane & 15)) * a.mp + 4 * (lane >> 4);
            const float *mcol = Ms + 4 * (lane >> 4) * MS + (lane & 15);
#pragma unroll
            for (int g0 = 0; g0 < NK; g0 += GB) {
                float4 av[GB];
#pragma unroll
                for (int u = 0; u < GB; ++u)
                    if (g0 + u < NK) av[u] = *reinterpret_cast<const float4 *>(vrow + 16 * (g0 + u));
#pragma unroll
                for (int u = 0; u < GB; ++u) {
                    if (g0 + u >= NK) break;
                    const float *mrow = mcol + 16 * (g0 + u) * MS;
                    v4f &d = (u & 1) ? d1 : d0;
                    d = __builtin_amdgcn_mfma_f32_16x16x4f32(av[u].x, mrow[0], d, 0, 0, 0);
                    d = __builtin_amdgcn_mfma_f32_16x16x4f32(av[u].y, mrow[MS], d, 0, 0, 0);
                    d = __builtin_amdgcn_mfma_f32_16x16x4f32(av[u].z, mrow[2 * MS], d, 0, 0, 0);
                    d = __builtin_amdgcn_mfma_f32_16x16x4f32(av[u].w, mrow[3 * MS], d, 0, 0, 0);
                }
            }
            return d0 + d1;
        };
        const int col = col0 + (lane & 15);
        const int64_t orow = int64_t(c) * r + col;     // output row (leaf, column)
        if constexpr (OUT != kOutF16S) {
            for (int rb = wave; rb < nrb; rb += 4) {
                const v4f d = compress_block(rb);
                const int k4 = rb * 16 + 4 * (lane >> 4);
                if (col >= r) continue;
                if constexpr (OUT == kOutF32) {
                    *reinterpret_cast<float4 *>(a.Mh + orow * kp + k4) = make_float4(d[0], d[1], d[2], d[3]);
                } else {
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        const uint16_t h = to_bf16(d[v]);
                        a.Mh16[orow * kp + k4 + v] = h;
                        a.Ml16[orow * kp + k4 + v] = to_bf16(d[v] - from_bf16(h));
                    }
                }
            }
        } else {
            // one power-of-two scale per (column, 64-rank chunk), max |x| 2^e in
            // [2^14, 2^15): the chunk's four row blocks are waves 0..3
            for (int ch = 0; ch < a.nchunk; ++ch) {
                const int rb = 4 * ch + wave;
                const v4f d = rb < nrb ? compress_block(rb) : v4f{0.f, 0.f, 0.f, 0.f};
                float mx = fmaxf(fmaxf(fabsf(d[0]), fabsf(d[1])), fmaxf(fabsf(d[2]), fabsf(d[3])));
                mx = fmaxf(mx, __shfl_xor(mx, 16, 64));
                mx = fmaxf(mx, __shfl_xor(mx, 32, 64));
                if (lane < 16) cmax[wave][lane] = mx;
                __syncthreads();
                mx = fmaxf(fmaxf(cmax[0][lane & 15], cmax[1][lane & 15]),
                           fmaxf(cmax[2][lane & 15], cmax[3][lane & 15]));
                const int e = mx > 0.f ? max(-126, min(126, 14 - ilogbf(mx))) : 0;
                if (rb < nrb && col < r) {
                    const int k4 = rb * 16 + 4 * (lane >> 4);
#pragma unroll
                    for (int v = 0; v < 4; ++v) a.Mh16[orow * kp + k4 + v] = to_f16(ldexpf(d[v], e));
                }
                if (wave == 0 && lane < 16 && col < r) a.Msinv[orow * a.nchunk + ch] = ldexpf(1.f, -e);
                __syncthreads();                  // cmax read before the next chunk writes it
            }
        }
        __syncthreads();                          // Ms complete for C; pool free
        // ---- C: translate into the parent (pencils; child octant uniform)
        const int oct = int(key & 7);
        float w[TPT][N];
#pragma unroll
        for (int u = 0; u < TPT; ++u) {
            const int task = tid + kThreads * u, j = task / NP, pnc = task % NP;
            const bool on = task < 16 * NP;
            float v[N];
#pragma unroll
            for (int k = 0; k < N; ++k) v[k] = on ? Ms[(pnc + NP * k) * MS + j] : 0.f;
            mode1<N, false>(cc, (oct >> 2) & 1, v, w[u]);
        }
#pragma unroll
        for (int u = 0; u < TPT; ++u) {
            const int task = tid + kThreads * u, j = task / NP, pnc = task % NP;
            if (task < 16 * NP)
#pragma unroll
                for (int k = 0; k < N; ++k) pool[j * m + pnc + NP * k] = w[u][k];
        }
        __syncthreads();
#pragma unroll
        for (int u = 0; u < TPT; ++u) {
            const int task = tid + kThreads * u, j = task / NP, pnc = task % NP;
            const int a1 = pnc % N, a3 = pnc / N;
            float v[N];
#pragma unroll
            for (int k = 0; k < N; ++k) v[k] = task < 16 * NP ? pool[j * m + a1 + N * k + NP * a3] : 0.f;
            mode1<N, false>(cc, (oct >> 1) & 1, v, w[u]);
        }
        __syncthreads();
#pragma unroll
        for (int u = 0; u < TPT; ++u) {
            const int task = tid + kThreads * u, j = task / NP, pnc = task % NP;
            const int a1 = pnc % N, a3 = pnc / N;
            if (task < 16 * NP)
#pragma unroll
                for (int k = 0; k < N; ++k) pool[j * m + a1 + N * k + NP * a3] = w[u][k];
        }
        __syncthreads();
#pragma unroll
        for (int u = 0; u < TPT; ++u) {
            const int task = tid + kThreads * u, j = task / NP, pnc = task % NP;
            float v[N], t[N];
#pragma unroll
            for (int k = 0; k < N; ++k) v[k] = task < 16 * NP ? pool[j * m + k + N * pnc] : 0.f;
            mode1<N, false>(cc, oct & 1, v, t);
#pragma unroll
            for (int k = 0; k < N; ++k) par[u][k] += t[k];
        }
    }
    // ---- the parent's coefficients (x-pencils: node k + N pencil)
#pragma unroll
    for (int u = 0; u < TPT; ++u) {
        const int task = tid + kThreads * u, j = task / NP, pnc = task % NP;
        if (task < 16 * NP && col0 + j < r) {
            float *out = a.Mpar + (int64_t(P) * r + col0 + j) * a.mp;
#pragma unroll
            for (int k = 0; k < N; ++k) out[k + N * pnc] = par[u][k];
        }
    }
    for (int g = tid; g < 16 * (a.mp - m); g += kThreads) {
        const int j = g / (a.mp - m);
        if (col0 + j < r) a.Mpar[(int64_t(P) * r + col0 + j) * a.mp + m + g % (a.mp - m)] = 0.f;
    }
}

// --------------------------------------------------------------- M2L ----
// One workgroup = one tile of up to 64 columns (target, rhs) of targets that
// share an octant, times 64 rows of the compressed rank.  For every slot
// j < 189 the octant fixes the transfer vector t; the sources Mh[k(a) + t]
// of the tile are staged in LDS and multiplied by C_t with
// v_mfma_f32_16x16x4f32 (each wave owns 16 rows x 64 columns).
// Lane layout of the 16x16x4 MFMA: A[i][k] from lane i + 16k, B[k][j] from
// lane j + 16k, D[i][j] in lane j + 16 (i / 4), register i % 4.  The K index
// of four consecutive MFMAs is permuted identically for A and B so each lane
// reads 4 consecutive K values with one 16-byte load.
constexpr int kM2LCols = 64;
constexpr int kMaskWords = (kSlots + 31) / 32;

// Visited slots of one workgroup: the set bits of the tile's mask within
// [jlo, jhi), in ascending order, as slot index and transfer-table index.
// Returns their number.  Called by all threads; ends with a barrier.
__device__ inline int tile_slot_list(const uint32_t *mask, int jlo, int jhi, const int32_t *slot_t,
                                     uint8_t *sl, int16_t *st) {
    uint32_t m[kMaskWords];
    int before[kMaskWords + 1];
    before[0] = 0;
#pragma unroll
    for (int w = 0; w < kMaskWords; ++w) {
        const int lo = max(jlo - 32 * w, 0), hi = min(jhi - 32 * w, 32);
        uint32_t range = 0;
        if (hi > lo) range = (hi - lo == 32 ? 0xffffffffu : ((1u << (hi - lo)) - 1u)) << lo;
        m[w] = mask[w] & range;
        before[w + 1] = before[w] + __popc(m[w]);
    }
    const int j = threadIdx.x;
    if (j < kSlots) {
        const int w = j >> 5, b = j & 31;
        if ((m[w] >> b) & 1u) {
            const int q = before[w] + __popc(m[w] & ((1u << b) - 1u));
            sl[q] = uint8_t(j);
            st[q] = int16_t(slot_t[j]);
        }
    }
    __syncthreads();
    return before[kMaskWords];
}

struct M2LLevel {
    const float *Mh;            // [C + 1][r][kp]: the extra cell C is all zeros
    float *Fh;                  // nsplit partial results, each [C][r][kp]
    const float *C32;
    const int32_t *itab;
    const int32_t *oct_cells;
    int kp;
    int64_t rows;               // C r: rows of one partial result (the zero cell is rows / r)
};

struct M2LArgs {
    M2LLevel lv[kMaxLevels];
    const int32_t *tiles;       // [ntiles][4]: level, octant, first in oct_cells, count
    const uint32_t *masks;      // [ntiles][kMaskWords]: slots with a source in the tile
    const int32_t *tables;      // slot_t[8][189] at offset 3 * 316
    int r, rc, tpt;
    int nsplit;                 // the 189 slots are split over this many workgroups
    int tile0;                  // first tile of this launch
    int ntiles;                 // tiles of this launch
    int xsplit;                 // splits pinned to XCDs (m2l_block_tile)
};

// Block index -> tile so that each XCD (blocks are dealt round-robin over
// the 8 XCDs) receives a contiguous run of tiles: neighbouring tiles share
// most of their sources, which then meet in the same L2.
__device__ inline int xcd_tile(int bid, int nblocks) {
    const int xcd = bid & 7, idx = bid >> 3;
    const int full = nblocks >> 3, rem = nblocks & 7;
    return xcd * full + min(xcd, rem) + idx;
}

// Block index -> (tile, slot split).  xsplit = 0: every XCD runs all splits
// of a contiguous run of tiles (xcd_tile).  xsplit = 1: XCD x runs split
// x % nsplit only (nsplit divides 8), and the 8 / nsplit XCDs of a split
// take contiguous runs of its tiles, so the operators of a split's slots
// (a 1 / nsplit share of the level's) are what its L2s hold.  The launch
// then has 8 ceil(ntiles nsplit / 8) blocks; false for the few past the end.
__device__ inline bool m2l_block_tile(int bid, int nblocks, int ntiles, int nsplit, int xsplit,
                                      int &tile, int &split) {
    if (!xsplit) {
        const int vb = xcd_tile(bid, nblocks);
        split = vb % nsplit;
        tile = vb / nsplit;
        return true;
    }
    const int x = bid & 7, idx = bid >> 3;
    const int G = 8 / nsplit, per = (ntiles + G - 1) / G;
    split = x % nsplit;
    tile = (x / nsplit) * per + idx;
    return tile < ntiles;
}

// Software-pipelined M2L.  A step is (slot j, K chunk kc of 64).  While the
// MFMAs of step s read LDS buffer s%2 and the C_t fragment held in
// registers, the loads of step s+1 (gathered sources and the next C_t rows)
// are already in flight into registers; they are written to the other LDS
// buffer after the MFMAs, followed by the step's only barrier.  The source
// index of slot j+3 is fetched during the last step of slot j into the
// three-deep ring entry that slot j no longer needs.
//
// Only the slots in which some target of the tile has a source are visited
// (a per-tile 189-bit mask made when the plan is built; a slot without a
// source would add exact zeros).  The slot range of a split is fixed in
// slot space, so which products land in which partial sum does not depend
// on how targets are grouped into tiles.  The last K chunk of a rank that
// is not a multiple of 64 issues only its nonzero 16-deep MFMA blocks, and
// waves whose 16 rows lie past the rank issue no MFMAs.
// FULL: every level of the launch has a rank padded to a whole 64-row
// group and every tile column is a right-hand side (r a multiple of the
// column tile), so no load needs a mask: a missing source reads the zero
// cell, and the per-element mask multiplies are gone.
template <int RW, bool FULL>
__global__ void __launch_bounds__(kThreads, 2) k_m2l(M2LArgs g) {
    static_assert(RW == 4 || RW == 2, "row waves");
    constexpr int RB = 4 / RW;          // 16-row blocks per wave
    constexpr int CB = RW;              // 16-column blocks per wave
    constexpr int ldb = 64 + 4;
    __shared__ float Bs[2][kM2LCols * ldb];
    __shared__ int32_t tgt[kM2LCols], srcs[3][kM2LCols];
    const int tid = threadIdx.x, lane = tid & 63;
    // wave-uniform, so that per-wave conditions compile to scalar branches
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    __shared__ uint8_t sl[kSlots];
    __shared__ int16_t st[kSlots];
    int tl, split;
    if (!m2l_block_tile(blockIdx.x, gridDim.x, g.ntiles, g.nsplit, g.xsplit, tl, split)) return;
    const int tix = g.tile0 + tl;
    const int4 tile = reinterpret_cast<const int4 *>(g.tiles)[tix];
    const M2LLevel &L = g.lv[tile.x];
    const int o = tile.y, start = tile.z, cnt = tile.w;
    const int kp = L.kp;
    if (int(blockIdx.y) * 64 >= kp) return;       // row group beyond this level's rank
    const float *Mh = L.Mh;
    const int32_t *itab = L.itab;
    const int r = g.r, rc = g.rc;
    const int rhs0 = blockIdx.z * rc;
    const int wr = wave % RW, wc = wave / RW;
    const int rowb = blockIdx.y * 64 + wr * 16 * RB;      // first row of the wave
    const int colb = wc * 16 * CB;                        // first column of the wave
    bool rok[RB];
    bool active = false;
#pragma unroll
    for (int b = 0; b < RB; ++b) {
        rok[b] = rowb + 16 * b < kp;
        active = active || rok[b];
    }
    const int nkc = (kp + 63) / 64;
    // visited slots of this split, compacted: index q runs over [0, jend)
    const int jbeg = 0;
    const int jend = tile_slot_list(g.masks + int64_t(tix) * kMaskWords, split * kSlots / g.nsplit,
                                    (split + 1) * kSlots / g.nsplit,
                                    g.tables + 3 * kNumT + o * kSlots, sl, st);
    const int nsteps = jend * nkc;
    (void)lane;

    if (tid < kM2LCols) {
        const int a = tid < cnt ? L.oct_cells[start + tid] : -1;
        tgt[tid] = a;
        for (int q = jbeg; q < min(jbeg + 3, jend); ++q)
            srcs[q % 3][tid] = a >= 0 ? itab[int64_t(a) * kSlots + sl[q]] : -1;
    }
    __syncthreads();

    // Per-thread share of one B chunk (64 columns x 16 float4): element
    // e = tid + 256 i is column e / 16, float4 e % 16.  Column -> (target
    // slot, rhs) is fixed for the whole tile, so all index math is hoisted.
    int bq[4], btl[4];
    int64_t boff[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int e = tid + i * kThreads;
        const int col = e >> 4;
        bq[i] = e & 15;
        btl[i] = col / rc;
        const int c = col - btl[i] * rc;
        boff[i] = (rhs0 + c < r) ? int64_t(rhs0 + c) * kp + 4 * bq[i] : -1;
    }
    // Loads are issued unconditionally from clamped in-bounds addresses and
    // masked afterwards: no branches, so the compiler never has to drain the
    // prefetches before the MFMAs of the current step.
    const int zc = int(L.rows / r);                      // the zero cell
    auto load_b = [&](int j, int kc, float4 (&breg)[4]) {
        const int lim = min(64, kp - kc * 64) / 4;   // float4 per column in this chunk
        const int32_t *sj = srcs[j % 3];
        int sc[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) sc[i] = sj[btl[i]];
        if constexpr (FULL) {
            (void)lim;
#pragma unroll
            for (int i = 0; i < 4; ++i)
                breg[i] = *reinterpret_cast<const float4 *>(
                    Mh + int64_t(sc[i] >= 0 ? sc[i] : zc) * r * kp + boff[i] + kc * 64);
        } else {
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const bool ok = sc[i] >= 0 && boff[i] >= 0 && bq[i] < lim;
                const float w = ok ? 1.f : 0.f;      // Mh is finite: 0 * v == 0
                const float4 v = *reinterpret_cast<const float4 *>(
                    Mh + (ok ? int64_t(sc[i]) * r * kp + boff[i] + kc * 64 : 0));
                breg[i] = make_float4(v.x * w, v.y * w, v.z * w, v.w * w);
            }
        }
    };
    auto store_b = [&](int buf, const float4 (&breg)[4]) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int e = tid + i * kThreads;
            *reinterpret_cast<float4 *>(&Bs[buf][(e >> 4) * ldb + 4 * bq[i]]) = breg[i];
        }
    };
    // rows past the rank read row 0 and are masked to zero
    int64_t arow[RB];
#pragma unroll
    for (int b = 0; b < RB; ++b)
        arow[b] = int64_t(rok[b] ? rowb + 16 * b + (lane & 15) : 0) * kp + 4 * (lane >> 4);
    auto load_a = [&](int j, int kc, float4 (&areg)[4 * RB]) {      // areg[b * 4 + kb]
        const int nkb = min(64, kp - kc * 64) / 16;
        const float *A = L.C32 + int64_t(st[j]) * kp * kp + kc * 64;
        if constexpr (FULL) {
            (void)nkb;
#pragma unroll
            for (int b = 0; b < RB; ++b)
#pragma unroll
                for (int kb = 0; kb < 4; ++kb)
                    areg[b * 4 + kb] = *reinterpret_cast<const float4 *>(A + arow[b] + 16 * kb);
        } else {
#pragma unroll
            for (int b = 0; b < RB; ++b)
#pragma unroll
                for (int kb = 0; kb < 4; ++kb) {
                    const bool ok = rok[b] && kb < nkb;    // wave-uniform
                    const float w = ok ? 1.f : 0.f;        // C32 is finite: 0 * v == 0
                    const float4 v = *reinterpret_cast<const float4 *>(A + arow[b] + (ok ? 16 * kb : 0));
                    areg[b * 4 + kb] = make_float4(v.x * w, v.y * w, v.z * w, v.w * w);
                }
        }
    };

    v4f acc[RB][CB];
#pragma unroll
    for (int b = 0; b < RB; ++b)
#pragma unroll
        for (int cb = 0; cb < CB; ++cb) acc[b][cb] = v4f{0.f, 0.f, 0.f, 0.f};
    float4 a0[4 * RB], a1[4 * RB];
    int32_t itab_next = -1;
    int j = jbeg, kc = 0;
    // One step: prefetch step s+1 (sources into breg, C_t rows into anxt,
    // the source index of slot j+3), multiply LDS buffer s%2 by acur, then
    // publish the prefetch.  Every prefetching step issues the same nine
    // unconditional loads per thread, so the compiler's wait counts stay
    // exact and the MFMAs never wait on the loads of the step they overlap.
    auto step = [&](auto more_c, int s, const float4 (&acur)[4 * RB], float4 (&anxt)[4 * RB]) {
        constexpr bool MORE = decltype(more_c)::value;
        int j1 = j, kc1 = kc + 1;
        if (kc1 == nkc) { kc1 = 0; ++j1; }
        const bool new_slot = MORE && kc1 == 0 && j + 3 < jend;
        float4 breg[4];                  // this step's prefetch of the next sources
        if constexpr (MORE) {
            load_b(j1, kc1, breg);
            load_a(j1, kc1, anxt);
            const int a = tgt[tid & 63];
            const int32_t v = itab[int64_t(a >= 0 ? a : 0) * kSlots + sl[min(j + 3, jend - 1)]];
            itab_next = a >= 0 ? v : -1;
        }
        // MFMA block: the 16-deep K blocks of this chunk that hold nonzero
        // rank (the zero-padded tail of a rank is skipped); waves whose rows
        // lie past the rank skip it entirely.  Both conditions are uniform.
        const int nkb = FULL ? 4 : (active ? min(64, kp - kc * 64) / 16 : 0);
        const float *B = Bs[s & 1] + (colb + (lane & 15)) * ldb + 4 * (lane >> 4);
#pragma unroll
        for (int kb = 0; kb < 4; ++kb) {
            if (kb >= nkb) break;
            float4 b4[CB];
#pragma unroll
            for (int cb = 0; cb < CB; ++cb)
                b4[cb] = *reinterpret_cast<const float4 *>(B + cb * 16 * ldb + 16 * kb);
#pragma unroll
            for (int b = 0; b < RB; ++b)
#pragma unroll
                for (int cb = 0; cb < CB; ++cb)
                    acc[b][cb] = __builtin_amdgcn_mfma_f32_16x16x4f32(acur[b * 4 + kb].x, b4[cb].x, acc[b][cb], 0, 0, 0);
#pragma unroll
            for (int b = 0; b < RB; ++b)
#pragma unroll
                for (int cb = 0; cb < CB; ++cb)
                    acc[b][cb] = __builtin_amdgcn_mfma_f32_16x16x4f32(acur[b * 4 + kb].y, b4[cb].y, acc[b][cb], 0, 0, 0);
#pragma unroll
            for (int b = 0; b < RB; ++b)
#pragma unroll
                for (int cb = 0; cb < CB; ++cb)
                    acc[b][cb] = __builtin_amdgcn_mfma_f32_16x16x4f32(acur[b * 4 + kb].z, b4[cb].z, acc[b][cb], 0, 0, 0);
#pragma unroll
            for (int b = 0; b < RB; ++b)
#pragma unroll
                for (int cb = 0; cb < CB; ++cb)
                    acc[b][cb] = __builtin_amdgcn_mfma_f32_16x16x4f32(acur[b * 4 + kb].w, b4[cb].w, acc[b][cb], 0, 0, 0);
        }
        if constexpr (MORE) {
            store_b((s + 1) & 1, breg);
            if (new_slot && tid < kM2LCols) srcs[j % 3][tid] = itab_next;
        }
        __syncthreads();
        j = j1;
        kc = kc1;
    };
    using yes = std::integral_constant<bool, true>;
    using no = std::integral_constant<bool, false>;
    if (nsteps > 0) {                    // uniform: no slot of this split has a source -> zeros
        float4 breg[4];
        load_b(jbeg, 0, breg);
        store_b(0, breg);
        load_a(jbeg, 0, a0);
        __syncthreads();
        int s = 0;
        for (; s + 2 < nsteps; s += 2) {
            step(yes{}, s, a0, a1);
            step(yes{}, s + 1, a1, a0);
        }
        if (s + 1 < nsteps) {
            step(yes{}, s, a0, a1);
            step(no{}, s + 1, a1, a0);
        } else {
            step(no{}, s, a0, a1);
        }
    }
    if (!active) return;
#pragma unroll
    for (int cb = 0; cb < CB; ++cb) {
        const int col = colb + cb * 16 + (lane & 15);
        const int tl = col / rc, c = col % rc;
        if (tl >= cnt || rhs0 + c >= r) continue;
        float *dst = L.Fh + split * L.rows * kp + (int64_t(tgt[tl]) * r + rhs0 + c) * kp + 4 * (lane >> 4);
#pragma unroll
        for (int b = 0; b < RB; ++b)
            if (rok[b])
                *reinterpret_cast<float4 *>(dst + rowb + 16 * b) =
                    make_float4(acc[b][cb][0], acc[b][cb][1], acc[b][cb][2], acc[b][cb][3]);
    }
}

// ----------------------------------------------- M2L, 16-bit operands ----
// Same tiling, slot split and software pipeline as k_m2l, on the gfx950
// 16x16x32 MFMAs.  Split-BF16: every operand is stored as hi + lo bf16
// halves and each product is hi*hi + hi*lo + lo*hi (FP32 accumulate).
// Scaled FP16: operands are fp16 scaled by powers of two (one per operator,
// one per source (cell, rhs, 64 ranks) block); each 64-rank chunk is
// accumulated from zero and folded into the FP32 result with the two
// inverse scales.  Lane layout of 16x16x32: A[i][k] from lane i + 16 (k/8),
// element k % 8; B[k][j] likewise; D as in 16x16x4.
struct M2LLevelLP {
    const uint16_t *Mh, *Ml;   // bf16 halves, or fp16 data in Mh  [rows][kp]
    const float *Msinv;        // fp16: inverse scales [rows][nchunk]
    float *Fh;                 // nsplit partial results [rows][kp]
    const uint16_t *Ch, *Cl;   // operator halves, or fp16 data in Ch  [316][kp][kp]
    const float *Cinv;         // fp16: operator inverse scales [316]
    const int32_t *itab;
    const int32_t *oct_cells;
    int kp;
    int64_t rows;
};

struct M2LArgsLP {
    M2LLevelLP lv[kMaxLevels];
    const int32_t *tiles;
    const uint32_t *masks;
    const int32_t *tables;
    int r, rc, tpt;
    int nsplit;
    int tile0;
    int ntiles;
    int xsplit;
};

typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef _Float16 v8h __attribute__((ext_vector_type(8)));
typedef float v16f __attribute__((ext_vector_type(16)));

template <int PREC>
__global__ void __launch_bounds__(kThreads, 2) k_m2l_lp(M2LArgsLP g) {
    constexpr bool X3 = PREC == BBFMM_M2L_BF16X3;
    constexpr int ldb = 64 + 8;                 // 144-byte rows: conflict-free 16-byte reads
    constexpr int NB = X3 ? 4 : 2;              // 16-byte source loads per thread per step
    constexpr int NA = X3 ? 4 : 2;              // 16-byte operator loads per lane per step
    __shared__ uint4 Bstore[2][X3 ? 2 : 1][kM2LCols * ldb / 8];
    __shared__ float Bsc[2][kM2LCols];
    __shared__ int32_t tgt[kM2LCols], srcs[3][kM2LCols];
    __shared__ uint8_t sl[kSlots];
    __shared__ int16_t st[kSlots];
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    int tl, split;
    if (!m2l_block_tile(blockIdx.x, gridDim.x, g.ntiles, g.nsplit, g.xsplit, tl, split)) return;
    const int tix = g.tile0 + tl;
    const int4 tile = reinterpret_cast<const int4 *>(g.tiles)[tix];
    const M2LLevelLP &L = g.lv[tile.x];
    const int o = tile.y, start = tile.z, cnt = tile.w;
    const int kp = L.kp;
    if (int(blockIdx.y) * 64 >= kp) return;
    const int32_t *itab = L.itab;
    const int r = g.r, rc = g.rc;
    const int rhs0 = blockIdx.z * rc;
    const int row0 = blockIdx.y * 64 + wave * 16;
    const bool active = row0 < kp;
    const int nkc = (kp + 63) / 64;
    const int jbeg = 0;
    const int jend = tile_slot_list(g.masks + int64_t(tix) * kMaskWords, split * kSlots / g.nsplit,
                                    (split + 1) * kSlots / g.nsplit,
                                    g.tables + 3 * kNumT + o * kSlots, sl, st);
    const int nsteps = jend * nkc;

    if (tid < kM2LCols) {
        const int a = tid < cnt ? L.oct_cells[start + tid] : -1;
        tgt[tid] = a;
        for (int q = jbeg; q < min(jbeg + 3, jend); ++q)
            srcs[q % 3][tid] = a >= 0 ? itab[int64_t(a) * kSlots + sl[q]] : -1;
    }
    __syncthreads();

    // source element e = tid + 256 i: column e / (2 NB), 16-byte piece e % (2 NB)
    // (X3: pieces 0..7 are hi, 8..15 lo; fp16: pieces 0..7)
    constexpr int PPC = X3 ? 16 : 8;            // pieces per column
    int bpart[NB], bsub[NB], btl[NB], bcol[NB];
    int64_t boff[NB];
#pragma unroll
    for (int i = 0; i < NB; ++i) {
        const int e = tid + i * kThreads;
        const int col = e / PPC, q = e % PPC;
        bcol[i] = col;
        bpart[i] = q >> 3;
        bsub[i] = q & 7;
        btl[i] = col / rc;
        const int c = col - btl[i] * rc;
        boff[i] = (rhs0 + c < r) ? int64_t(rhs0 + c) * kp + 8 * bsub[i] : -1;
    }
    // per-column scale of the staged chunk (fp16): column tid & 63
    const int scol = tid & 63, stl = scol / rc, sc_c = scol - (scol / rc) * rc;
    const int nchunk = nkc;

    auto load_b = [&](int j, int kc, uint4 *breg, float &bscale) {
        const int lim = min(64, kp - kc * 64) / 8;     // 16-byte pieces per half-column
        const int32_t *sj = srcs[j % 3];
#pragma unroll
        for (int i = 0; i < NB; ++i) {
            const int scl = sj[btl[i]];
            const bool ok = scl >= 0 && boff[i] >= 0 && bsub[i] < lim;
            const uint16_t *base = bpart[i] ? L.Ml : L.Mh;
            const uint4 v = *reinterpret_cast<const uint4 *>(
                base + (ok ? int64_t(scl) * r * kp + boff[i] + kc * 64 : 0));
            const uint32_t w = ok ? 0xffffffffu : 0u;
            breg[i] = make_uint4(v.x & w, v.y & w, v.z & w, v.w & w);
        }
        if constexpr (!X3) {
            const int scl = sj[stl];
            const bool ok = scl >= 0 && rhs0 + sc_c < r;
            const float v = L.Msinv[ok ? (int64_t(scl) * r + rhs0 + sc_c) * nchunk + kc : 0];
            bscale = ok ? v : 0.f;
        }
    };
    auto store_b = [&](int buf, const uint4 *breg, float bscale) {
#pragma unroll
        for (int i = 0; i < NB; ++i)
            Bstore[buf][bpart[i]][(bcol[i] * ldb + 8 * bsub[i]) / 8] = breg[i];
        if constexpr (!X3) Bsc[buf][scol] = bscale;   // four waves store the same value
    };
    const int64_t arow = int64_t(active ? row0 + (lane & 15) : 0) * kp + 8 * (lane >> 4);
    auto load_a = [&](int j, int kc, uint4 *areg) {
        const int nks = min(64, kp - kc * 64) / 32;
        const int64_t base = int64_t(st[j]) * kp * kp + arow + kc * 64;
#pragma unroll
        for (int i = 0; i < NA; ++i) {
            const int ks = i & 1;
            const bool ok = active && ks < nks;
            const uint16_t *C = (X3 && i >= 2) ? L.Cl : L.Ch;
            const uint4 v = *reinterpret_cast<const uint4 *>(C + (ok ? base + 32 * ks : 0));
            const uint32_t w = ok ? 0xffffffffu : 0u;
            areg[i] = make_uint4(v.x & w, v.y & w, v.z & w, v.w & w);
        }
    };

    v4f acc[4];
    for (int cb = 0; cb < 4; ++cb) acc[cb] = v4f{0.f, 0.f, 0.f, 0.f};
    uint4 breg[NB], a0[NA], a1[NA];
    float bscale = 0.f;
    int32_t itab_next = -1;
    int j = jbeg, kc = 0;
    auto step = [&](auto more_c, int s, const uint4 *acur, uint4 *anxt) {
        constexpr bool MORE = decltype(more_c)::value;
        int j1 = j, kc1 = kc + 1;
        if (kc1 == nkc) { kc1 = 0; ++j1; }
        const bool new_slot = MORE && kc1 == 0 && j + 3 < jend;
        float cinv = 0.f;
        if constexpr (!X3) cinv = L.Cinv[st[j]];
        if constexpr (MORE) {
            load_b(j1, kc1, breg, bscale);
            load_a(j1, kc1, anxt);
            const int a = tgt[tid & 63];
            const int32_t v = itab[int64_t(a >= 0 ? a : 0) * kSlots + sl[min(j + 3, jend - 1)]];
            itab_next = a >= 0 ? v : -1;
        }
        // 32-deep K blocks holding nonzero rank; none for waves past the rank
        const int nks = active ? min(64, kp - kc * 64) / 32 : 0;
        const uint4 *Bh = Bstore[s & 1][0];
        const int bbase = ((lane & 15) * ldb + 8 * (lane >> 4)) / 8;
        if constexpr (X3) {
            const uint4 *Bl = Bstore[s & 1][1];
#pragma unroll
            for (int ks = 0; ks < 2; ++ks) {
                if (ks >= nks) break;
                v8bf bh[4], bl[4];
#pragma unroll
                for (int cb = 0; cb < 4; ++cb) {
                    bh[cb] = __builtin_bit_cast(v8bf, Bh[bbase + (cb * 16 * ldb + 32 * ks) / 8]);
                    bl[cb] = __builtin_bit_cast(v8bf, Bl[bbase + (cb * 16 * ldb + 32 * ks) / 8]);
                }
                const v8bf ah = __builtin_bit_cast(v8bf, acur[ks]);
                const v8bf al = __builtin_bit_cast(v8bf, acur[2 + ks]);
#pragma unroll
                for (int cb = 0; cb < 4; ++cb)
                    acc[cb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bh[cb], acc[cb], 0, 0, 0);
#pragma unroll
                for (int cb = 0; cb < 4; ++cb)
                    acc[cb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bl[cb], acc[cb], 0, 0, 0);
#pragma unroll
                for (int cb = 0; cb < 4; ++cb)
                    acc[cb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bh[cb], acc[cb], 0, 0, 0);
            }
        } else if (nks > 0) {
            v4f part[4];
#pragma unroll
            for (int cb = 0; cb < 4; ++cb) part[cb] = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int ks = 0; ks < 2; ++ks) {
                if (ks >= nks) break;
                const v8h a16 = __builtin_bit_cast(v8h, acur[ks]);
#pragma unroll
                for (int cb = 0; cb < 4; ++cb) {
                    const v8h b16 = __builtin_bit_cast(v8h, Bh[bbase + (cb * 16 * ldb + 32 * ks) / 8]);
                    part[cb] = __builtin_amdgcn_mfma_f32_16x16x32_f16(a16, b16, part[cb], 0, 0, 0);
                }
            }
#pragma unroll
            for (int cb = 0; cb < 4; ++cb) {
                const float f = Bsc[s & 1][cb * 16 + (lane & 15)] * cinv;
                acc[cb] += part[cb] * f;
            }
        }
        if constexpr (MORE) {
            store_b((s + 1) & 1, breg, bscale);
            if (new_slot && tid < kM2LCols) srcs[j % 3][tid] = itab_next;
        }
        __syncthreads();
        j = j1;
        kc = kc1;
    };
    using yes = std::integral_constant<bool, true>;
    using no = std::integral_constant<bool, false>;
    if (nsteps > 0) {
        load_b(jbeg, 0, breg, bscale);
        store_b(0, breg, bscale);
        load_a(jbeg, 0, a0);
        __syncthreads();
        int s = 0;
        for (; s + 2 < nsteps; s += 2) {
            step(yes{}, s, a0, a1);
            step(yes{}, s + 1, a1, a0);
        }
        if (s + 1 < nsteps) {
            step(yes{}, s, a0, a1);
            step(no{}, s + 1, a1, a0);
        } else {
            step(no{}, s, a0, a1);
        }
    }
    if (!active) return;
    for (int cb = 0; cb < 4; ++cb) {
        const int col = cb * 16 + (lane & 15);
        const int tl = col / rc, c = col % rc;
        if (tl < cnt && rhs0 + c < r) {
            float *dst = L.Fh + split * L.rows * kp +
                         (int64_t(tgt[tl]) * r + rhs0 + c) * kp + row0 + 4 * (lane >> 4);
            *reinterpret_cast<float4 *>(dst) = make_float4(acc[cb][0], acc[cb][1], acc[cb][2], acc[cb][3]);
        }
    }
}

// ------------------------------ M2L, 16-bit operands, parent blocks ----
// For blocks of right-hand sides the tile kernel above gathers every source
// block once per (target, slot) pair.  Here a workgroup takes the (up to
// eight) children of one parent cell as its targets.  Their interaction
// lists all lie among the 6 x 6 x 6 children of the parent's neighbours
// (the halo; position h = k(b) - 2 k(parent) + 2 per axis), and a halo cell
// b interacts with every child a it is not adjacent to, with transfer
// vector t = h - 2 - o(a) (o(a): the child's offset, the octant bits).  So
// each occupied halo cell's compressed multipoles are staged in LDS once per
// 32-rank chunk and serve all children that see them (about seven on a full
// grid), while the operator rows C_t come from L2 (316 operators per
// level).  Wave w owns children 2w and 2w+1: RB 16-row blocks of the rank
// times CB 16-column blocks of right-hand sides for each, as 16x16x32
// MFMAs; with W32 (RB = 2, CB = 2 or 4) the same 32 rows x 16 CB columns
// are 32x32x16 MFMAs instead (half as many instructions, each operand
// fragment serving twice the outputs).  The sum over the
// halo is complete inside the workgroup (one partial result).  The loads of
// the next step -- the staged source chunk and the wave's operator rows --
// are issued before the MFMAs of the current one.
struct M2LBlockArgs {
    const uint16_t *Mh, *Ml;   // level operands [C][r][kp] (bf16 hi / lo, or fp16 in Mh)
    const float *Msinv;        // fp16: inverse block scales [C][r][nchunk]
    float *Fh;                 // [C][r][kp]
    const uint16_t *Ch, *Cl;   // operators [316][kp][kp]
    const float *Cinv;         // fp16: operator inverse scales [316]
    const int32_t *itab;       // [C][189]
    const uint64_t *keys;      // level keys (child octant = key & 7)
    const int32_t *pcb, *pce;  // children of each parent (level above)
    const int32_t *t_slot;     // [8][316]: slot of transfer vector t for an octant, -1
    int kp, r;
};

// compact index of t in {-3..3}^3 minus {-1..1}^3 (ascending (tx+3) + 7(ty+3) + 49(tz+3))
__device__ inline int t_compact(int tx, int ty, int tz) {
    const int code = (tx + 3) + 7 * (ty + 3) + 49 * (tz + 3);
    int inner = 0;                            // codes of {-1..1}^3 below this one
    for (int z = 2; z <= 4; ++z)
        for (int y = 2; y <= 4; ++y)
            for (int x = 2; x <= 4; ++x) inner += (x + 7 * y + 49 * z) < code;
    return code - inner;
}

template <int PREC, int RB, int CB, bool W32>
__global__ void __launch_bounds__(kThreads, 2) k_m2l_blk(M2LBlockArgs g) {
    static_assert(!W32 || (RB == 2 && (CB == 2 || CB == 4)), "32x32 blocks: 32 rows, 32 or 64 columns");
    constexpr bool X3 = PREC == BBFMM_M2L_BF16X3;
    constexpr int C32 = W32 ? CB / 2 : 1;       // 32-column blocks (W32)
    constexpr int COLS = 16 * CB;
    constexpr int ldb = 32 + 8;                 // 80-byte column rows (32 ranks + pad)
    constexpr int PPC = X3 ? 8 : 4;             // 16-byte pieces per column (hi + lo for X3)
    constexpr int NB = (COLS * PPC + kThreads - 1) / kThreads;
    constexpr int NH = 216;                     // halo positions
    __shared__ uint4 Bstore[2][X3 ? 2 : 1][COLS * ldb / 8];
    __shared__ float Bsc[2][COLS];
    __shared__ int32_t hb[NH];                  // compacted: source cell
    __shared__ uint8_t hmask[NH];               // children that interact with it
    __shared__ int16_t htix[NH][8];             // their transfer-vector indices
    __shared__ int wcount[4];
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int P = xcd_tile(blockIdx.x, gridDim.x);
    const int c0 = g.pcb[P], nchild = g.pce[P] - c0;
    const int kp = g.kp, r = g.r;
    const int row0 = blockIdx.y * 16 * RB;
    const int rhs0 = blockIdx.z * COLS;
    const int nkc = (kp + 31) / 32;             // 32-deep rank chunks (kp is a multiple of 32)
    const int nc64 = (kp + 63) / 64;            // fp16 scales are per 64 ranks
    int oct[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) oct[i] = i < nchild ? int(g.keys[c0 + i] & 7u) : 0;

    // ---- the halo: occupied positions that some child interacts with
    int my_b = -1;
    unsigned my_m = 0;
    int16_t my_t[8];
    const int hx = tid % 6, hy = (tid / 6) % 6, hz = tid / 36;
#pragma unroll
    for (int i = 0; i < 8; ++i) {             // unrolled: the arrays stay in registers
        my_t[i] = -1;
        if (tid >= NH || i >= nchild) continue;
        const int o = oct[i];
        const int tx = hx - 2 - (o & 1), ty = hy - 2 - ((o >> 1) & 1), tz = hz - 2 - (o >> 2);
        if (max(abs(tx), max(abs(ty), abs(tz))) < 2) continue;         // adjacent: near field
        const int ti = t_compact(tx, ty, tz);
        const int slot = g.t_slot[o * kNumT + ti];
        const int src = slot >= 0 ? g.itab[int64_t(c0 + i) * kSlots + slot] : -1;
        if (src < 0) continue;
        my_b = src;                           // the same cell for every child that sees it
        my_m |= 1u << i;
        my_t[i] = int16_t(ti);
    }
    const bool have = my_m != 0u;
    const uint64_t bal = __ballot(have);
    const int before = __popcll(bal & ((uint64_t(1) << lane) - 1));
    if (lane == 0) wcount[wave] = __popcll(bal);
    __syncthreads();
    int off = 0;
    for (int w = 0; w < wave; ++w) off += wcount[w];
    const int nh = wcount[0] + wcount[1] + wcount[2] + wcount[3];
    if (have) {
        const int q = off + before;
        hb[q] = my_b;
        hmask[q] = uint8_t(my_m);
#pragma unroll
        for (int i = 0; i < 8; ++i) htix[q][i] = my_t[i];
    }
    __syncthreads();
    if (row0 >= kp) return;                     // uniform: a row group past the rank

    // staged piece e = tid + 256 i: column e / PPC, 16-byte piece e % PPC
    int bpart[NB], bsub[NB], bcol[NB];
    int64_t boff[NB];
#pragma unroll
    for (int i = 0; i < NB; ++i) {
        const int e = tid + i * kThreads;
        const int col = e / PPC, q = e % PPC;
        bcol[i] = col;
        bpart[i] = q >> 2;
        bsub[i] = q & 3;
        boff[i] = (e < COLS * PPC && rhs0 + col < r) ? int64_t(rhs0 + col) * kp + 8 * bsub[i] : -1;
    }
    const int scol = tid % COLS;
    auto load_b = [&](int s, uint4 *breg, float &bscale) {
        const int h = s / nkc, kc = s - (s / nkc) * nkc;
        const int b = hb[h];
#pragma unroll
        for (int i = 0; i < NB; ++i) {
            const bool ok = boff[i] >= 0;
            const uint16_t *base = bpart[i] ? g.Ml : g.Mh;
            const uint4 v = *reinterpret_cast<const uint4 *>(
                base + (ok ? int64_t(b) * r * kp + boff[i] + kc * 32 : 0));
            const uint32_t w = ok ? 0xffffffffu : 0u;
            breg[i] = make_uint4(v.x & w, v.y & w, v.z & w, v.w & w);
        }
        if constexpr (!X3) {
            const bool ok = rhs0 + scol < r;
            const float v = g.Msinv[ok ? (int64_t(b) * r + rhs0 + scol) * nc64 + kc / 2 : 0];
            bscale = ok ? v : 0.f;
        }
    };
    auto store_b = [&](int buf, const uint4 *breg, float bscale) {
#pragma unroll
        for (int i = 0; i < NB; ++i)
            if (bcol[i] < COLS) Bstore[buf][bpart[i]][(bcol[i] * ldb + 8 * bsub[i]) / 8] = breg[i];
        if constexpr (!X3) if (tid < COLS) Bsc[buf][scol] = bscale;
    };

    v4f acc[2][RB][CB];
    v16f acc32[2][C32];
#pragma unroll
    for (int u = 0; u < 2; ++u) {
#pragma unroll
        for (int rb = 0; rb < RB; ++rb)
#pragma unroll
            for (int cb = 0; cb < CB; ++cb) acc[u][rb][cb] = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int c2 = 0; c2 < C32; ++c2)
#pragma unroll
            for (int e = 0; e < 16; ++e) acc32[u][c2][e] = 0.f;
    }
    const int nsteps = nh * nkc;
    // operator rows of this wave's two children for one step, prefetched one
    // step ahead like the sources: 16x16x32 -- RB 16-row blocks, lane holds
    // row (lane & 15), ranks 8 (lane >> 4) .. + 7 of the 32-rank chunk;
    // W32 -- two 16-deep halves ks (in the rb slot), lane holds row
    // (lane & 31), ranks 16 ks + 8 (lane >> 5) .. + 7
    constexpr int NP = X3 ? 2 : 1;
    uint4 acur[2][RB][NP], anxt[2][RB][NP];
    float ccur[2] = {0.f, 0.f}, cnxt[2] = {0.f, 0.f};
    auto load_a = [&](int st, uint4 (&a)[2][RB][NP], float (&cv)[2]) {
        const int h = st / nkc, kc = st - (st / nkc) * nkc;
        const unsigned hm = hmask[h];
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            const int i = 2 * wave + u;
            const bool valid = (hm >> i) & 1u;                  // wave-uniform
            const int ti = valid ? int(htix[h][i]) : 0;
            if constexpr (!X3) cv[u] = valid ? g.Cinv[ti] : 0.f;
#pragma unroll
            for (int rb = 0; rb < RB; ++rb) {
                const int64_t cbase = int64_t(ti) * kp * kp + kc * 32 +
                                      (W32 ? 16 * rb + 8 * (lane >> 5) : 8 * (lane >> 4));
                const int row = W32 ? row0 + (lane & 31) : row0 + rb * 16 + (lane & 15);
                const bool ok = valid && row < kp;
                const int64_t o = ok ? cbase + int64_t(row) * kp : 0;
                const uint32_t w = ok ? 0xffffffffu : 0u;
                uint4 v = make_uint4(0u, 0u, 0u, 0u);
                if (valid) v = *reinterpret_cast<const uint4 *>(g.Ch + o);
                a[u][rb][0] = make_uint4(v.x & w, v.y & w, v.z & w, v.w & w);
                if constexpr (X3) {
                    if (valid) v = *reinterpret_cast<const uint4 *>(g.Cl + o);
                    a[u][rb][NP - 1] = make_uint4(v.x & w, v.y & w, v.z & w, v.w & w);
                }
            }
        }
    };
    uint4 breg[NB];
    float bscale = 0.f;
    if (nsteps > 0) {
        load_b(0, breg, bscale);
        load_a(0, acur, ccur);
        store_b(0, breg, bscale);
    }
    __syncthreads();
    const int bbase = ((lane & 15) * ldb + 8 * (lane >> 4)) / 8;
    for (int s = 0; s < nsteps; ++s) {
        const bool more = s + 1 < nsteps;
        if (more) {
            load_b(s + 1, breg, bscale);
            load_a(s + 1, anxt, cnxt);
        }
        const int h = s / nkc;
        const unsigned hm = hmask[h];
        const uint4 *Bh = Bstore[s & 1][0];
        if constexpr (W32) {
            const int b32 = ((lane & 31) * ldb + 8 * (lane >> 5)) / 8;
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                const int i = 2 * wave + u;
                if (!((hm >> i) & 1u)) continue;                // wave-uniform
                v16f part[C32];
                if constexpr (!X3) {
#pragma unroll
                    for (int c2 = 0; c2 < C32; ++c2)
#pragma unroll
                        for (int e = 0; e < 16; ++e) part[c2][e] = 0.f;
                }
#pragma unroll
                for (int c2 = 0; c2 < C32; ++c2)
#pragma unroll
                    for (int ks = 0; ks < 2; ++ks) {
                        const int bi = b32 + (c2 * 32 * ldb + 16 * ks) / 8;
                        if constexpr (X3) {
                            const v8bf bh = __builtin_bit_cast(v8bf, Bh[bi]);
                            const v8bf bl = __builtin_bit_cast(v8bf, Bstore[s & 1][1][bi]);
                            const v8bf a_h = __builtin_bit_cast(v8bf, acur[u][ks][0]);
                            const v8bf a_l = __builtin_bit_cast(v8bf, acur[u][ks][NP - 1]);
                            acc32[u][c2] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a_h, bh, acc32[u][c2], 0, 0, 0);
                            acc32[u][c2] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a_h, bl, acc32[u][c2], 0, 0, 0);
                            acc32[u][c2] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a_l, bh, acc32[u][c2], 0, 0, 0);
                        } else {
                            part[c2] = __builtin_amdgcn_mfma_f32_32x32x16_f16(
                                __builtin_bit_cast(v8h, acur[u][ks][0]), __builtin_bit_cast(v8h, Bh[bi]),
                                part[c2], 0, 0, 0);
                        }
                    }
                if constexpr (!X3) {
#pragma unroll
                    for (int c2 = 0; c2 < C32; ++c2) {
                        const float f = Bsc[s & 1][c2 * 32 + (lane & 31)] * ccur[u];
#pragma unroll
                        for (int e = 0; e < 16; ++e) acc32[u][c2][e] += part[c2][e] * f;
                    }
                }
            }
        } else
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            const int i = 2 * wave + u;
            if (!((hm >> i) & 1u)) continue;                    // wave-uniform
            v4f part[RB][CB];
            if constexpr (!X3) {
#pragma unroll
                for (int rb = 0; rb < RB; ++rb)
#pragma unroll
                    for (int cb = 0; cb < CB; ++cb) part[rb][cb] = v4f{0.f, 0.f, 0.f, 0.f};
            }
#pragma unroll
            for (int cb = 0; cb < CB; ++cb) {
                const uint4 braw = Bh[bbase + cb * 16 * ldb / 8];
                if constexpr (X3) {
                    const v8bf bh = __builtin_bit_cast(v8bf, braw);
                    const v8bf bl = __builtin_bit_cast(v8bf, Bstore[s & 1][1][bbase + cb * 16 * ldb / 8]);
#pragma unroll
                    for (int rb = 0; rb < RB; ++rb) {
                        const v8bf a_h = __builtin_bit_cast(v8bf, acur[u][rb][0]);
                        const v8bf a_l = __builtin_bit_cast(v8bf, acur[u][rb][NP - 1]);
                        acc[u][rb][cb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a_h, bh, acc[u][rb][cb], 0, 0, 0);
                        acc[u][rb][cb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a_h, bl, acc[u][rb][cb], 0, 0, 0);
                        acc[u][rb][cb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a_l, bh, acc[u][rb][cb], 0, 0, 0);
                    }
                } else {
                    const v8h b16 = __builtin_bit_cast(v8h, braw);
#pragma unroll
                    for (int rb = 0; rb < RB; ++rb)
                        part[rb][cb] = __builtin_amdgcn_mfma_f32_16x16x32_f16(
                            __builtin_bit_cast(v8h, acur[u][rb][0]), b16, part[rb][cb], 0, 0, 0);
                }
            }
            if constexpr (!X3) {
#pragma unroll
                for (int cb = 0; cb < CB; ++cb) {
                    const float f = Bsc[s & 1][cb * 16 + (lane & 15)] * ccur[u];
#pragma unroll
                    for (int rb = 0; rb < RB; ++rb) acc[u][rb][cb] += part[rb][cb] * f;
                }
            }
        }
        if (more) store_b((s + 1) & 1, breg, bscale);
        __syncthreads();
        if (more) {
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                ccur[u] = cnxt[u];
#pragma unroll
                for (int rb = 0; rb < RB; ++rb)
#pragma unroll
                    for (int q = 0; q < NP; ++q) acur[u][rb][q] = anxt[u][rb][q];
            }
        }
    }
    if constexpr (W32) {
        // 32x32 accumulator: element 4 q + e is row 8 q + 4 (lane >> 5) + e,
        // column lane & 31 of the block
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            const int i = 2 * wave + u;
            if (i >= nchild) continue;
#pragma unroll
            for (int c2 = 0; c2 < C32; ++c2) {
                const int c = rhs0 + c2 * 32 + (lane & 31);
                if (c >= r) continue;
                float *dst = g.Fh + (int64_t(c0 + i) * r + c) * kp + row0 + 4 * (lane >> 5);
#pragma unroll
                for (int q = 0; q < 4; ++q)
                    *reinterpret_cast<float4 *>(dst + 8 * q) =
                        make_float4(acc32[u][c2][4 * q], acc32[u][c2][4 * q + 1], acc32[u][c2][4 * q + 2],
                                    acc32[u][c2][4 * q + 3]);
            }
        }
        return;
    }
#pragma unroll
    for (int u = 0; u < 2; ++u) {
        const int i = 2 * wave + u;
        if (i >= nchild) continue;
#pragma unroll
        for (int cb = 0; cb < CB; ++cb) {
            const int c = rhs0 + cb * 16 + (lane & 15);
            if (c >= r) continue;
            float *dst = g.Fh + (int64_t(c0 + i) * r + c) * kp + 4 * (lane >> 4);
#pragma unroll
            for (int rb = 0; rb < RB; ++rb) {
                const int row = row0 + rb * 16;
                if (row < kp)
                    *reinterpret_cast<float4 *>(dst + row) =
                        make_float4(acc[u][rb][cb][0], acc[u][rb][cb][1], acc[u][rb][cb][2], acc[u][rb][cb][3]);
            }
        }
    }
}

// --------------------------------------------------------- L2P + P2P ----
// One wave per work item (leaf a, first target t0, log2 S): the wave holds
// T = 64 / S targets, each spread over S consecutive lanes ("sub-lanes").
// The sources of all neighbour leaves are copied into LDS in as few passes
// as fit (x, y, z, sigma packed in one 16-byte record, zero-padded to a
// multiple of the inner loop's step -- 8 S records for one right-hand side,
// 4 S otherwise -- so the loop is uniform and unrolled; padding records have
// sigma = 0 and a finite kernel value).  Sub-lane s takes
// records s, s + S, ... and the i3 planes s, s + S, ... of the L2P sum; the
// S partial sums of a target are added by a fixed butterfly of cross-lane
// shuffles, so results are reproducible.
template <int RC>
struct P2PCap {   // records per LDS pass: a multiple of 64, about 8-17 KB of LDS per wave
    static constexpr int value = RC == 1 ? 512 : (RC <= 4 ? 256 : (RC <= 16 ? 128 : 64));
};

template <int KID, int RC, int S>
__device__ inline void p2p_records(const float4 *sp, const float (*ss)[RC > 1 ? RC - 1 : 1],
                                   int npad, int sub, float x, float y, float z, float *acc) {
    if constexpr (RC == 1) {
        float a0 = 0.f, a1 = 0.f;
        for (int u = 0; u < npad; u += 8 * S) {
#pragma unroll
            for (int v = 0; v < 8; v += 2) {
                const float4 q0 = sp[u + v * S + sub];
                const float4 q1 = sp[u + (v + 1) * S + sub];
                const float k0 = kernel_eval<KID>(x - q0.x, y - q0.y, z - q0.z);
                const float k1 = kernel_eval<KID>(x - q1.x, y - q1.y, z - q1.z);
                a0 += k0 * q0.w;
                a1 += k1 * q1.w;
            }
        }
        acc[0] += a0 + a1;
    } else {
        for (int u = 0; u < npad; u += 4 * S) {
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int jj = u + v * S + sub;
                const float4 q = sp[jj];
                const float k = kernel_eval<KID>(x - q.x, y - q.y, z - q.z);
                acc[0] += k * q.w;
#pragma unroll
                for (int c = 1; c < RC; ++c) acc[c] += k * ss[jj][c - 1];
            }
        }
    }
}

template <int KID, int RC>
__global__ void __launch_bounds__(64)
k_p2p(const float *xs, const float *ys, const float *zs, const int32_t *sb_leaf, const int32_t *pe,
      const int32_t *te, const int32_t *nbr_off, const int32_t *nbr_idx, const uint64_t *keys,
      const int32_t *perm, const int32_t *work, int nwork, const float *sig_s, int r, float cs,
      const float *FL, int mp, Geo geo, ChebConst cc, float *phi) {
    constexpr int CAP = P2PCap<RC>::value;
    __shared__ float4 sp[CAP];                        // x, y, z, sigma of the first rhs
    __shared__ float ss[CAP][RC > 1 ? RC - 1 : 1];    // remaining rhs
    __shared__ int32_t nb_end[64], nb_src[64];        // neighbour chunk: running end, first point
    const int lane = threadIdx.x;
    // grid-stride over the work items: a launch of fewer workgroups than items
    // keeps the near field to a share of the chip (overlapped schedule)
    for (int item = blockIdx.x; item < nwork; item += gridDim.x) {
        const int a = work[3 * item], t0 = work[3 * item + 1];
        const int lgS = min(work[3 * item + 2], 4);   // at most 16 sub-lanes
        const int S = 1 << lgS, sub = lane & (S - 1);
        const int rhs0 = blockIdx.y * RC;
        const int nr = min(RC, r - rhs0);
        const int i = t0 + (lane >> lgS);
        const bool valid = i < te[a];
        const float x = valid ? xs[i] : 0.f, y = valid ? ys[i] : 0.f, z = valid ? zs[i] : 0.f;
        const float xc = x * cs, yc = y * cs, zc = z * cs;   // kernel coordinates
        float acc[RC];
#pragma unroll
        for (int c = 0; c < RC; ++c) acc[c] = 0.f;
        // The neighbour leaves' records form one sequence (list order, points
        // in tree order), cut into LDS passes of CAP records.  A chunk of up
        // to 64 neighbours is described by one lane each (first point and
        // record count, prefix-summed across the wave), so a pass is staged
        // with independent loads: record e of the chunk belongs to the first
        // neighbour whose running end exceeds e (binary search in LDS).
        const int q0 = nbr_off[a], q1 = nbr_off[a + 1];
        for (int qc = q0; qc < q1; qc += 64) {
            int sb = 0, cnt = 0;
            if (qc + lane < q1) {
                const int b = nbr_idx[qc + lane];
                sb = sb_leaf[b];
                cnt = pe[b] - sb;
            }
            int inc = cnt;
#pragma unroll
            for (int d = 1; d < 64; d <<= 1) {
                const int t = __shfl_up(inc, d, 64);
                if (lane >= d) inc += t;
            }
            const int total = __shfl(inc, 63, 64);
            __syncthreads();                     // the previous chunk's table is consumed
            nb_end[lane] = inc;
            nb_src[lane] = sb - (inc - cnt);     // record e of this neighbour is point nb_src + e
            for (int base = 0; base < total; base += CAP) {
                const int n = min(CAP, total - base);
                __syncthreads();                 // table visible, previous pass consumed
                constexpr int KS = CAP / 64;
                int src[KS];
#pragma unroll
                for (int k = 0; k < KS; ++k) {          // all searches, then all loads
                    const int e = base + lane + 64 * k;
                    int j = 0;
#pragma unroll
                    for (int st = 32; st > 0; st >>= 1)
                        if (nb_end[j + st - 1] <= e) j += st;
                    src[k] = e < base + n ? nb_src[min(j, 63)] + e : -1;
                }
                float4 rec[KS];
#pragma unroll
                for (int k = 0; k < KS; ++k) {
                    const int q = max(src[k], 0);
                    rec[k] = make_float4(xs[q], ys[q], zs[q], sig_s[int64_t(q) * r + rhs0]);
                }
#pragma unroll
                for (int k = 0; k < KS; ++k) {
                    const float w = src[k] >= 0 ? 1.f : 0.f, wc = w * cs;
                    sp[lane + 64 * k] = make_float4(rec[k].x * wc, rec[k].y * wc, rec[k].z * wc, rec[k].w * w);
                }
                if constexpr (RC > 1) {
#pragma unroll
                    for (int k = 0; k < KS; ++k) {
                        const float *sg = sig_s + int64_t(max(src[k], 0)) * r + rhs0;
                        const float w = src[k] >= 0 ? 1.f : 0.f;
#pragma unroll
                        for (int c = 1; c < RC; ++c) ss[lane + 64 * k][c - 1] = c < nr ? sg[c] * w : 0.f;
                    }
                }
                // records n .. CAP are zero; the loop below reads up to a multiple of its step
                const int G = RC == 1 ? 8 * S : 4 * S;
                const int npad = min(CAP, (n + G - 1) / G * G);
                __syncthreads();
                switch (lgS) {
                case 0: p2p_records<KID, RC, 1>(sp, ss, npad, sub, xc, yc, zc, acc); break;
                case 1: p2p_records<KID, RC, 2>(sp, ss, npad, sub, xc, yc, zc, acc); break;
                case 2: p2p_records<KID, RC, 4>(sp, ss, npad, sub, xc, yc, zc, acc); break;
                case 3: p2p_records<KID, RC, 8>(sp, ss, npad, sub, xc, yc, zc, acc); break;
                default: p2p_records<KID, RC, 16>(sp, ss, npad, sub, xc, yc, zc, acc); break;
                }
            }
        }
        if (FL != nullptr && valid) {
            const int n = cc.n;
            const uint64_t key = keys[a];
            float l[3][kMaxOrder];
            const float p[3] = {x, y, z};
            for (int d = 0; d < 3; ++d) {
                float chi, clo;
                center_pair(geo.lo[d], compact3(key >> d), geo.h, chi, clo);
                lagrange(cc, local_coord(p[d], chi, clo, geo.inv_h), l[d]);
            }
            for (int c = 0; c < RC; ++c) {
                if (c >= nr) break;
                const float *f = FL + (int64_t(a) * r + rhs0 + c) * mp;
                float sacc = 0.f;
                for (int i3 = sub; i3 < n; i3 += S) {
                    float s2 = 0.f;
                    for (int i2 = 0; i2 < n; ++i2) {
                        float s1 = 0.f;
                        for (int i1 = 0; i1 < n; ++i1) s1 += l[0][i1] * f[(i3 * n + i2) * n + i1];
                        s2 += l[1][i2] * s1;
                    }
                    sacc += l[2][i3] * s2;
                }
                acc[c] += sacc;
            }
        }
        for (int msk = 1; msk < S; msk <<= 1) {
#pragma unroll
            for (int c = 0; c < RC; ++c) acc[c] += __shfl_xor(acc[c], msk, 64);
        }
        if (valid && sub == 0) {
            float *out = phi + int64_t(perm[i]) * r + rhs0;
#pragma unroll
            for (int c = 0; c < RC; ++c)
                if (c < nr) out[c] = acc[c];
        }
        __syncthreads();                  // LDS of this item is consumed
    }
}

// ----------------------------------------- packed per-lane P2P ----
// One right-hand side.  A work item (leaf a, first target t0, S, tpl, G)
// holds G groups of tpl consecutive targets; lane l serves group l / S as
// sub-lane l mod S, so that any leaf size fills the wave: S need not be a
// power of two and each lane evaluates tpl targets against every record it
// reads (the record is loaded once from LDS for all of them).  Sub-lane s
// takes records s, s + S, ... of each LDS pass, stored contiguously for it;
// a pass holds a multiple of the loop step U S (U = 8 records per step for
// one target per lane, 4 otherwise; zero records pad it; they have sigma =
// 0 and a finite kernel value).  The S partial sums of a target are added
// in sub-lane order through LDS, so results are reproducible.  The kernel
// writes the near field only; k_l2p adds the far field after it.
constexpr int kPackCap = 512;                 // records per LDS pass, at most

template <int KID, int TPL>
__device__ inline void p2p_pack_item(const float *xs, const float *ys, const float *zs,
                                     const int32_t *sb_leaf, const int32_t *pe, const int32_t *te,
                                     const int32_t *nbr_off, const int32_t *nbr_idx,
                                     const int32_t *perm, const float *sig_s, int ld, float cs,
                                     int a, int t0, int cnt_t, int S, int G, float4 *sp,
                                     int32_t *nb_end, int32_t *nb_src, float *red, float *phi) {
    constexpr int KS = kPackCap / 64;
    const int lane = threadIdx.x;
    const int g = lane / S, sub = lane - g * S;
    const int tend = min(te[a], t0 + cnt_t);   // this item's targets only (a leaf may have several)
    float x[TPL], y[TPL], z[TPL], acc[TPL];
#pragma unroll
    for (int k = 0; k < TPL; ++k) {
        const int i = t0 + g * TPL + k;
        const bool ok = g < G && i < tend;
        x[k] = ok ? xs[i] * cs : 0.f;
        y[k] = ok ? ys[i] * cs : 0.f;
        z[k] = ok ? zs[i] * cs : 0.f;
        acc[k] = 0.f;
    }
    float acc1 = 0.f;                          // second chain of the single-target form
    constexpr int U = TPL == 1 ? 8 : 4;        // records per sub-lane per loop step
    const int step = U * S;
    const int pass = kPackCap / step * step;   // records per pass: whole loop steps
    const int rcp = (65536 + S - 1) / S;       // e / S = (e rcp) >> 16 for e < 600, S <= 16
    const int q0 = nbr_off[a], q1 = nbr_off[a + 1];
    for (int qc = q0; qc < q1; qc += 64) {
        int sb = 0, cnt = 0;
        if (qc + lane < q1) {
            const int b = nbr_idx[qc + lane];
            sb = sb_leaf[b];
            cnt = pe[b] - sb;
        }
        int inc = cnt;
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            const int tv = __shfl_up(inc, d, 64);
            if (lane >= d) inc += tv;
        }
        const int total = __shfl(inc, 63, 64);
        __syncthreads();                       // the previous chunk's table is consumed
        nb_end[lane] = inc;
        nb_src[lane] = sb - (inc - cnt);       // record e of this neighbour is point nb_src + e
        for (int base = 0; base < total; base += pass) {
            const int n = min(pass, total - base);
            __syncthreads();                   // table visible, previous pass consumed
            // record e of the pass goes to row e mod S, column e / S of an
            // S x (M + 1) table (M = npad / S): each sub-lane then reads its
            // records at consecutive addresses, and the odd row pitch keeps
            // the S rows' reads on different banks.  Staged in two halves
            // (fewer registers live beside the targets' accumulators).
            const int npad = (n + step - 1) / step * step;   // <= pass <= kPackCap
            const int M = npad / S;
            constexpr int KH = KS / 2;
#pragma unroll 1
            for (int h = 0; h < 2; ++h) {
                int src[KH];
#pragma unroll
                for (int k = 0; k < KH; ++k) {
                    const int e = base + lane + 64 * (h * KH + k);
                    int j = 0;
#pragma unroll
                    for (int st = 32; st > 0; st >>= 1)
                        if (nb_end[j + st - 1] <= e) j += st;
                    src[k] = e < base + n ? nb_src[min(j, 63)] + e : -1;
                }
                float4 rec[KH];
#pragma unroll
                for (int k = 0; k < KH; ++k) {
                    const int q = max(src[k], 0);
                    rec[k] = make_float4(xs[q], ys[q], zs[q], sig_s[int64_t(q) * ld]);
                }
#pragma unroll
                for (int k = 0; k < KH; ++k) {
                    const int e = lane + 64 * (h * KH + k);
                    if (e < npad) {
                        const int col = (e * rcp) >> 16, row = e - col * S;
                        const float w = src[k] >= 0 ? 1.f : 0.f, wc = w * cs;
                        sp[row * (M + 1) + col] =
                            make_float4(rec[k].x * wc, rec[k].y * wc, rec[k].z * wc, rec[k].w * w);
                    }
                }
            }
            __syncthreads();
            const float4 *mine = sp + sub * (M + 1);
            for (int u = 0; u < M; u += U) {
#pragma unroll
                for (int v = 0; v < U; ++v) {
                    const float4 q = mine[u + v];
#pragma unroll
                    for (int k = 0; k < TPL; ++k) {
                        const float kv = kernel_eval<KID>(x[k] - q.x, y[k] - q.y, z[k] - q.z);
                        if (TPL == 1 && (v & 1)) acc1 += kv * q.w;
                        else acc[k] += kv * q.w;
                    }
                }
            }
        }
    }
    acc[0] += acc1;
#pragma unroll
    for (int k = 0; k < TPL; ++k) red[k * 64 + lane] = acc[k];
    __syncthreads();
    if (g < G && sub == 0) {
#pragma unroll
        for (int k = 0; k < TPL; ++k) {
            const int i = t0 + g * TPL + k;
            if (i < tend) {
                float sum = 0.f;
                for (int j = 0; j < S; ++j) sum += red[k * 64 + lane + j];
                phi[perm[i]] = sum;
            }
        }
    }
    __syncthreads();                           // LDS of this item is consumed
}

template <int KID>
__global__ void __launch_bounds__(64)
k_p2p_pack(const float *xs, const float *ys, const float *zs, const int32_t *sb_leaf, const int32_t *pe,
           const int32_t *te, const int32_t *nbr_off, const int32_t *nbr_idx, const int32_t *perm,
           const int32_t *work, int nwork, const float *sig_s, int ld, float cs, float *phi) {
    __shared__ float4 sp[kPackCap + 16];        // S rows of pitch npad / S + 1
    __shared__ int32_t nb_end[64], nb_src[64];
    __shared__ float red[4 * 64];
    for (int item = blockIdx.x; item < nwork; item += gridDim.x) {
        const int a = work[3 * item], t0 = work[3 * item + 1], code = work[3 * item + 2];
        const int S = code & 31, tpl = (code >> 5) & 7, G = (code >> 8) & 127, cnt = code >> 15;
        switch (tpl) {
        case 1:
            p2p_pack_item<KID, 1>(xs, ys, zs, sb_leaf, pe, te, nbr_off, nbr_idx, perm, sig_s, ld, cs,
                                  a, t0, cnt, S, G, sp, nb_end, nb_src, red, phi);
            break;
        case 2:
            p2p_pack_item<KID, 2>(xs, ys, zs, sb_leaf, pe, te, nbr_off, nbr_idx, perm, sig_s, ld, cs,
                                  a, t0, cnt, S, G, sp, nb_end, nb_src, red, phi);
            break;
        default:
            p2p_pack_item<KID, 4>(xs, ys, zs, sb_leaf, pe, te, nbr_off, nbr_idx, perm, sig_s, ld, cs,
                                  a, t0, cnt, S, G, sp, nb_end, nb_src, red, phi);
            break;
        }
    }
}

// -------------------------------------------- L2P + P2P on MFMA ----
// For a block of right-hand sides the near field is a product,
// phi[i][c] += sum_j K(x_i, y_j) sigma[j][c].  One wave takes up to 64
// targets of a leaf (four 16-row blocks) and 16 NCB columns.  Each
// v_mfma_f32_16x16x4f32 multiplies a 16 x 4 block of kernel values, which
// lane i + 16 k evaluates itself (target i, source k) straight into its A
// operand, by the 4 x 16 block of the sources' sigma staged in LDS, so one
// kernel evaluation serves 16 NCB columns.  The far field (L2P) is the
// same product with the Lagrange basis S[i][node] in place of K and the
// leaf's local expansion F in place of sigma, accumulated first into the
// same registers.  A column's arithmetic does not depend on the other
// columns, on NCB or on r.
template <int NCB>
struct P2PMfmaCap {   // source records per LDS pass (coordinates + NCB x 16 sigma)
    static constexpr int value = NCB == 1 ? 128 : 64;
};

template <int KID, int NCB, int NRB>
__global__ void __launch_bounds__(64)
k_p2p_mfma(const float *xs, const float *ys, const float *zs, const int32_t *sb_leaf,
           const int32_t *pe, const int32_t *te, const int32_t *nbr_off, const int32_t *nbr_idx,
           const uint64_t *keys, const int32_t *perm, const int32_t *work, const float *sig_s, int ld, int r, float cs,
           const float *FL, int mp, Geo geo, ChebConst cc, float *phi) {
    constexpr int CW = 16 * NCB;            // columns of this wave
    constexpr int SST = CW == 16 ? 16 : CW + 16;   // = 16 mod 32: rows k, k+1 on disjoint banks
    constexpr int CAP = P2PMfmaCap<NCB>::value;
    constexpr int RPL = CAP / 64;           // staged records per lane (coordinates)
    constexpr int QPR = CW / 4;             // 16-byte sigma pieces per record
    constexpr int SPL = CAP * QPR / 64;     // sigma pieces per lane
    static_assert(CAP * SST >= 4 * 16 * 3 * kMaxOrder, "Lagrange values share the sigma buffer");
    __shared__ float4 sp[CAP];
    __shared__ __align__(16) float ss[CAP * SST];
    __shared__ int32_t sidx[CAP];
    __shared__ int16_t ntab[kMaxOrder * kMaxOrder * kMaxOrder];
    // Lagrange values of the targets, [4][16][3 kMaxOrder]; used before the
    // first staging pass, whose barrier retires them
    float (*Ls)[16][3 * kMaxOrder] = reinterpret_cast<float (*)[16][3 * kMaxOrder]>(ss);
    const int lane = threadIdx.x, row = lane & 15, kq = lane >> 4;
    const int a = work[2 * blockIdx.x], t0 = work[2 * blockIdx.x + 1];
    const int tend = te[a];
    const int col0 = blockIdx.y * CW;
    float tx[NRB], ty[NRB], tz[NRB];
#pragma unroll
    for (int rb = 0; rb < NRB; ++rb) {
        const int ti = t0 + 16 * rb + row;
        const int tc = ti < tend ? ti : t0;   // rows past the leaf repeat a target; not written
        tx[rb] = xs[tc];
        ty[rb] = ys[tc];
        tz[rb] = zs[tc];
    }
    v4f acc[NRB][NCB];
#pragma unroll
    for (int rb = 0; rb < NRB; ++rb)
#pragma unroll
        for (int cb = 0; cb < NCB; ++cb) acc[rb][cb] = v4f{0.f, 0.f, 0.f, 0.f};

    if (FL != nullptr) {
        const int n = cc.n, m = n * n * n;
        for (int i = lane; i < m; i += 64)
            ntab[i] = int16_t((i % n) | ((i / n) % n) << 4 | (i / (n * n)) << 8);
        if (kq == 0) {
            const uint64_t key = keys[a];
            float chi[3], clo[3];
            for (int d = 0; d < 3; ++d) center_pair(geo.lo[d], compact3(key >> d), geo.h, chi[d], clo[d]);
            for (int rb = 0; rb < NRB; ++rb) {
                const float p3[3] = {tx[rb], ty[rb], tz[rb]};
                for (int d = 0; d < 3; ++d) {
                    float l[kMaxOrder];
                    lagrange(cc, local_coord(p3[d], chi[d], clo[d], geo.inv_h), l);
                    for (int q = 0; q < n; ++q) Ls[rb][row][d * kMaxOrder + q] = l[q];
                }
            }
        }
        __syncthreads();
        const float *Fa = FL + int64_t(a) * r * mp;
        int64_t fcol[NCB];
        float fw[NCB];
#pragma unroll
        for (int cb = 0; cb < NCB; ++cb) {
            const int c = col0 + cb * 16 + row;
            fw[cb] = c < r ? 1.f : 0.f;        // F is finite: 0 * v == 0
            fcol[cb] = int64_t(c < r ? c : 0) * mp;
        }
        // U node steps per batch: their F loads are issued together
        constexpr int U = 4;
        for (int nb = 0; nb < m; nb += 4 * U) {
            float bv[U][NCB];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int node = nb + 4 * u + kq;
                const int nd = node < m ? node : 0;
#pragma unroll
                for (int cb = 0; cb < NCB; ++cb) bv[u][cb] = Fa[fcol[cb] + nd] * fw[cb];
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int node = nb + 4 * u + kq;
                const bool nok = node < m;
                const int code = ntab[nok ? node : 0];
                const int k1 = code & 15, k2 = (code >> 4) & 15, k3 = code >> 8;
                float sv[NRB];
#pragma unroll
                for (int rb = 0; rb < NRB; ++rb) {
                    const float *L3 = Ls[rb][row];
                    const float v = L3[k1] * L3[kMaxOrder + k2] * L3[2 * kMaxOrder + k3];
                    sv[rb] = nok ? v : 0.f;
                }
#pragma unroll
                for (int rb = 0; rb < NRB; ++rb)
#pragma unroll
                    for (int cb = 0; cb < NCB; ++cb)
                        acc[rb][cb] = __builtin_amdgcn_mfma_f32_16x16x4f32(sv[rb], bv[u][cb], acc[rb][cb], 0, 0, 0);
            }
        }
    }

    // Near field over the neighbour leaves, staged in LDS passes of CAP
    // records.  Passes are software-pipelined: the global loads of pass p+1
    // are in flight in registers while pass p is multiplied out of LDS.
    const int q1 = nbr_off[a + 1];
    int q = nbr_off[a], off = 0;
    float cx[RPL], cy[RPL], cz[RPL];
    float4 sv[SPL];
    // source indices of the next pass into sidx, then its loads into registers
    auto fetch = [&]() -> int {
        int cnt_all = 0;
        while (q < q1 && cnt_all < CAP) {
            const int b = nbr_idx[q];
            const int sb = sb_leaf[b] + off, cnt = min(pe[b] - sb, CAP - cnt_all);
            for (int e = lane; e < cnt; e += 64) sidx[cnt_all + e] = sb + e;
            cnt_all += cnt;
            if (sb + cnt == pe[b]) { ++q; off = 0; } else { off += cnt; }
        }
        __syncthreads();
#pragma unroll
        for (int u = 0; u < RPL; ++u) {
            const int e = lane + 64 * u;
            const int src = e < cnt_all ? sidx[e] : 0;
            cx[u] = xs[src];
            cy[u] = ys[src];
            cz[u] = zs[src];
        }
#pragma unroll
        for (int u = 0; u < SPL; ++u) {
            const int g = lane + 64 * u, e = g / QPR, part = g % QPR;
            const int src = e < cnt_all ? sidx[e] : 0;
            sv[u] = *reinterpret_cast<const float4 *>(sig_s + int64_t(src) * ld + col0 + 4 * part);
        }
        return cnt_all;
    };
    // the fetched records into LDS; records past cnt (the pad to a multiple of 4) are zero
    auto publish = [&](int cnt) {
#pragma unroll
        for (int u = 0; u < RPL; ++u) {
            const int e = lane + 64 * u;
            sp[e] = e < cnt ? make_float4(cx[u] * cs, cy[u] * cs, cz[u] * cs, 0.f)
                            : make_float4(0.f, 0.f, 0.f, 0.f);
        }
#pragma unroll
        for (int u = 0; u < SPL; ++u) {
            const int g = lane + 64 * u, e = g / QPR, part = g % QPR;
            const float w = e < cnt ? 1.f : 0.f;       // sigma is finite: 0 * v == 0
            *reinterpret_cast<float4 *>(&ss[e * SST + 4 * part]) =
                make_float4(sv[u].x * w, sv[u].y * w, sv[u].z * w, sv[u].w * w);
        }
    };
    __syncthreads();                    // Lagrange values (in ss) are consumed
#pragma unroll
    for (int rb = 0; rb < NRB; ++rb) {  // kernel coordinates from here on
        tx[rb] *= cs;
        ty[rb] *= cs;
        tz[rb] *= cs;
    }
    int cnt = q < q1 ? fetch() : 0;
    while (cnt > 0) {
        publish(cnt);
        __syncthreads();
        const int npad = (cnt + 3) & ~3;
        cnt = q < q1 ? fetch() : 0;     // loads of the next pass overlap the products below
        // LDS operands one step ahead (the last step re-reads its own)
        float4 sq_n = sp[kq];
        float bv_n[NCB];
#pragma unroll
        for (int cb = 0; cb < NCB; ++cb) bv_n[cb] = ss[kq * SST + cb * 16 + row];
        for (int s0 = 0; s0 < npad; s0 += 4) {
            const float4 sq = sq_n;
            float bv[NCB];
#pragma unroll
            for (int cb = 0; cb < NCB; ++cb) bv[cb] = bv_n[cb];
            const int nx = min(s0 + 4, npad - 4) + kq;
            sq_n = sp[nx];
#pragma unroll
            for (int cb = 0; cb < NCB; ++cb) bv_n[cb] = ss[nx * SST + cb * 16 + row];
            float kv[NRB];
#pragma unroll
            for (int rb = 0; rb < NRB; ++rb)
                kv[rb] = kernel_eval<KID>(tx[rb] - sq.x, ty[rb] - sq.y, tz[rb] - sq.z);
#pragma unroll
            for (int rb = 0; rb < NRB; ++rb)
#pragma unroll
                for (int cb = 0; cb < NCB; ++cb)
                    acc[rb][cb] = __builtin_amdgcn_mfma_f32_16x16x4f32(kv[rb], bv[cb], acc[rb][cb], 0, 0, 0);
        }
        __syncthreads();                // this pass is consumed before the next publish
    }
    // D[i][j] sits in lane j + 16 (i / 4), register i % 4
#pragma unroll
    for (int rb = 0; rb < NRB; ++rb) {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int ti = t0 + 16 * rb + 4 * kq + v;
            if (ti >= tend) continue;
            float *out = phi + int64_t(perm[ti]) * r;
#pragma unroll
            for (int cb = 0; cb < NCB; ++cb) {
                const int c = col0 + cb * 16 + row;
                if (c < r) out[c] = acc[rb][cb][v];
            }
        }
    }
}

// ---------------------------------------------------------------- L2P ----
// Far field added to phi, one thread per point (tree order):
// phi[perm[i]][c] += sum_node S[i][node] F[leaf(i)][c][node], with the
// separable Lagrange product summed x fastest.  Runs after the near field
// has written phi (the overlapped schedule).  The local expansions of the
// leaves that a workgroup's points fall in are staged in LDS (one padded
// row per leaf, so the lanes of different leaves read different banks);
// a workgroup whose points span more leaves than fit reads them from
// global memory instead.
constexpr int kL2PLdsFloats = 8192;

template <int N>
__device__ inline float l2p_sum(const float *f, const float (*l)[N]) {
    float sacc = 0.f;
#pragma unroll
    for (int i3 = 0; i3 < N; ++i3) {
        float s2 = 0.f;
#pragma unroll
        for (int i2 = 0; i2 < N; ++i2) {
            float s1 = 0.f;
#pragma unroll
            for (int i1 = 0; i1 < N; ++i1) s1 += l[0][i1] * f[(i3 * N + i2) * N + i1];
            s2 += l[1][i2] * s1;
        }
        sacc += l[2][i3] * s2;
    }
    return sacc;
}

template <int N>
__global__ void __launch_bounds__(kThreads)
k_l2p(const float *xs, const float *ys, const float *zs, const int32_t *pleaf, const uint64_t *keys,
      const int32_t *perm, int64_t npts, int64_t n_out, int r, const float *FL, int mp, Geo geo,
      ChebConst cc, float *phi) {
    constexpr int m = N * N * N, RS = m | 1;          // LDS row stride (odd)
    __shared__ float fs[kL2PLdsFloats];
    const int64_t i0 = int64_t(blockIdx.x) * kThreads;
    const int64_t i = i0 + threadIdx.x;
    const int64_t ilast = min(i0 + kThreads, npts) - 1;
    const int afirst = pleaf[i0], alast = pleaf[ilast];
    const int nl = alast - afirst + 1;
    const bool staged = int64_t(nl) * RS <= kL2PLdsFloats;      // uniform
    const bool active = i < npts;
    const int a = active ? pleaf[i] : afirst;
    float l[3][N];
    if (active) {
        const uint64_t key = keys[a];
        const float p3[3] = {xs[i], ys[i], zs[i]};
        for (int d = 0; d < 3; ++d) {
            float chi, clo;
            center_pair(geo.lo[d], compact3(key >> d), geo.h, chi, clo);
            lagrange_t<N>(cc, local_coord(p3[d], chi, clo, geo.inv_h), l[d]);
        }
    }
    for (int c = 0; c < r; ++c) {
        float sacc = 0.f;
        if (staged) {
            __syncthreads();                  // previous column consumed
            for (int e = threadIdx.x; e < nl * m; e += kThreads) {
                const int la = e / m, node = e - la * m;
                fs[la * RS + node] = FL[(int64_t(afirst + la) * r + c) * mp + node];
            }
            __syncthreads();
            if (active) sacc = l2p_sum<N>(fs + (a - afirst) * RS, l);
        } else if (active) {
            sacc = l2p_sum<N>(FL + (int64_t(a) * r + c) * mp, l);
        }
        if (active && perm[i] < n_out) phi[int64_t(perm[i]) * r + c] += sacc;   // targets only
    }
}

// ------------------------------------------ level-adaptive tree stages ----
// Chebyshev node i of a cell (key on a level of half-width h), in kernel
// coordinates (times the kernel's coordinate scale cs).
template <int N>
__device__ inline void node_coords(const ChebConst &cc, const float *lo, uint64_t key, float h,
                                   float cs, int i, float *out) {
    const int id[3] = {i % N, (i / N) % N, i / (N * N)};
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        float chi, clo;
        center_pair(lo[d], compact3(key >> d), h, chi, clo);
        out[d] = (chi + __fmaf_rn(h, cc.s[id[d]], clo)) * cs;
    }
}

// P2L over the X lists of one level: F[cell][c][i] += sum over the points
// y_j of the cell's X leaves of K(x*_i, y_j) sigma_j[c], x*_i the cell's
// Chebyshev nodes (the local expansion holds the far field at the nodes).
// One wave per (cell with an X list, RC columns); lanes own nodes, sources
// are staged 64 at a time, and each kernel value serves the RC columns.
template <int N, int KID, int RC>
__global__ void __launch_bounds__(64)
k_p2l(const int32_t *xcells, const int32_t *xoff, const int32_t *xleaf, const int32_t *lpb,
      const int32_t *lpe, const uint64_t *keys, const float *xs, const float *ys, const float *zs,
      const float *sig_s, int ld, Geo geo, ChebConst cc, float cs, int r, int mp, float *F) {
    constexpr int m = N * N * N, Q = (m + 63) / 64;
    __shared__ float4 sp[64];
    __shared__ float sv[64][RC];
    const int lane = threadIdx.x;
    const int cell = xcells[blockIdx.x], c0 = blockIdx.y * RC;
    const int nr = min(RC, r - c0);
    const uint64_t key = keys[cell];
    float nx[Q][3], acc[Q][RC];
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        node_coords<N>(cc, geo.lo, key, geo.h, cs, min(lane + 64 * q, m - 1), nx[q]);
#pragma unroll
        for (int c = 0; c < RC; ++c) acc[q][c] = 0.f;
    }
    for (int e = xoff[cell]; e < xoff[cell + 1]; ++e) {
        const int a = xleaf[e], b = lpb[a], en = lpe[a];
        for (int p0 = b; p0 < en; p0 += 64) {
            const int np = min(64, en - p0);
            __syncthreads();                       // previous chunk consumed
            if (lane < np) {
                const int j = p0 + lane;
                sp[lane] = make_float4(xs[j] * cs, ys[j] * cs, zs[j] * cs, 0.f);
#pragma unroll
                for (int c = 0; c < RC; ++c) sv[lane][c] = c < nr ? sig_s[int64_t(j) * ld + c0 + c] : 0.f;
            }
            __syncthreads();
            for (int j = 0; j < np; ++j) {
                const float4 y = sp[j];
                float sg[RC];
#pragma unroll
                for (int c = 0; c < RC; ++c) sg[c] = sv[j][c];
#pragma unroll
                for (int q = 0; q < Q; ++q) {
                    const float kv = kernel_eval<KID>(nx[q][0] - y.x, nx[q][1] - y.y, nx[q][2] - y.z);
#pragma unroll
                    for (int c = 0; c < RC; ++c) acc[q][c] += kv * sg[c];
                }
            }
        }
    }
#pragma unroll
    for (int c = 0; c < RC; ++c) {
        float *f = F + (int64_t(cell) * r + c0 + (c < nr ? c : 0)) * mp;
#pragma unroll
        for (int q = 0; q < Q; ++q)
            if (c < nr && lane + 64 * q < m) f[lane + 64 * q] += acc[q][c];
    }
}

// P2L as a product on FP32 MFMA for blocks of 16 right-hand sides:
// F[cell][c][node] += sum_j K(x*_node, y_j) sigma_j[c], lane i + 16 k
// evaluating node i of a 16-row block against point 4 s + k into its A
// operand, sigma as B.  One wave per (cell with an X list, 16 columns),
// nodes in chunks of 64 (four 16-row blocks); the X leaves' points are
// staged 64 at a time (padded to a multiple of 4 with zero sigma).
template <int N, int KID>
__global__ void __launch_bounds__(64)
k_p2l_mfma(const int32_t *xcells, const int32_t *xoff, const int32_t *xleaf, const int32_t *lpb,
           const int32_t *lpe, const uint64_t *keys, const float *xs, const float *ys, const float *zs,
           const float *sig_s, int ld, Geo geo, ChebConst cc, float cs, int r, int mp, float *F) {
    constexpr int m = N * N * N;
    __shared__ float4 sp[64];
    __shared__ float ss[64][16];
    const int lane = threadIdx.x, row = lane & 15, kq = lane >> 4;
    const int cell = xcells[blockIdx.x], c0 = blockIdx.y * 16;
    const int nr = min(16, r - c0);
    const uint64_t key = keys[cell];
    for (int n0 = 0; n0 < m; n0 += 64) {
        float nx[4][3];
#pragma unroll
        for (int rb = 0; rb < 4; ++rb)
            node_coords<N>(cc, geo.lo, key, geo.h, cs, min(n0 + 16 * rb + row, m - 1), nx[rb]);
        v4f acc[4];
#pragma unroll
        for (int rb = 0; rb < 4; ++rb) acc[rb] = v4f{0.f, 0.f, 0.f, 0.f};
        for (int e = xoff[cell]; e < xoff[cell + 1]; ++e) {
            const int a = xleaf[e], b = lpb[a], en = lpe[a];
            for (int p0 = b; p0 < en; p0 += 64) {
                const int np = min(64, en - p0), npad = (np + 3) & ~3;
                __syncthreads();                   // previous points consumed
                {
                    const int j = p0 + (lane < np ? lane : 0);
                    sp[lane] = make_float4(xs[j] * cs, ys[j] * cs, zs[j] * cs, 0.f);
                }
                for (int g = lane; g < 64 * 16; g += 64) {
                    const int jj = g >> 4, c = g & 15;
                    ss[jj][c] = (jj < np && c < nr) ? sig_s[int64_t(p0 + jj) * ld + c0 + c] : 0.f;
                }
                __syncthreads();
                for (int s0 = 0; s0 < npad; s0 += 4) {
                    const float4 y = sp[s0 + kq];
                    const float bv = ss[s0 + kq][row];
#pragma unroll
                    for (int rb = 0; rb < 4; ++rb) {
                        const float kv = kernel_eval<KID>(nx[rb][0] - y.x, nx[rb][1] - y.y, nx[rb][2] - y.z);
                        acc[rb] = __builtin_amdgcn_mfma_f32_16x16x4f32(kv, bv, acc[rb], 0, 0, 0);
                    }
                }
            }
        }
        // D[i][j] sits in lane j + 16 (i / 4), register i % 4: node i, column j
        if (row < nr) {
            float *f = F + (int64_t(cell) * r + c0 + row) * mp;
#pragma unroll
            for (int rb = 0; rb < 4; ++rb)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int node = n0 + 16 * rb + 4 * kq + v;
                    if (node < m) f[node] += acc[rb][v];
                }
        }
    }
}

// Per-level arrays of a plan over a level-adaptive tree, by value.
struct LevelExp {
    const float *F[kMaxLevels];      // local expansions (levels >= 2)
    const float *M[kMaxLevels];      // multipole expansions (levels >= 2)
    const uint64_t *keys[kMaxLevels];
    float h[kMaxLevels], inv_h[kMaxLevels];
};

// The far field at the points of every leaf of a level-adaptive tree, added
// to phi after the near field: L2P from the leaf's local expansion (leaves on
// levels >= 2) and M2P over its W list, phi(x) += sum_i K(x, y*_i) M_A[i]
// with y*_i the Chebyshev nodes of cell A.  One wave per (leaf, RC
// columns); lanes own targets; a W cell's node coordinates and its RC
// columns of coefficients are staged in LDS, and each kernel value serves
// the RC columns.  The leaf's local expansion is read at wave-uniform
// addresses.
template <int N, int KID, int RC>
__global__ void __launch_bounds__(64)
k_leaf_far(const int32_t *lpb, const int32_t *lpe, const uint64_t *lkey, const int32_t *llev,
           const int32_t *lcell, const int32_t *woff, const int32_t *wlev, const int32_t *wcell,
           LevelExp X, const float *xs, const float *ys, const float *zs, const int32_t *perm,
           Geo geo, ChebConst cc, float cs, int r, int mp, float *phi) {
    constexpr int m = N * N * N, Q = (m + 63) / 64;
    __shared__ float4 nd[64 * Q];        // a W cell's node coordinates (kernel units)
    __shared__ float ms[64 * Q][RC];     // ... and its coefficients, RC columns
    const int lane = threadIdx.x;
    const int q = blockIdx.x, c0 = blockIdx.y * RC;
    const int nr = min(RC, r - c0);
    const int lv = llev[q], b = lpb[q], e = lpe[q];
    const uint64_t key = lkey[q];
    const int w0 = woff[q], w1 = woff[q + 1];
    for (int p0 = b; p0 < e; p0 += 64) {
        const int i = p0 + lane;
        const bool valid = i < e;
        const int ii = valid ? i : b;
        const float x = xs[ii], y = ys[ii], z = zs[ii];
        float acc[RC];
#pragma unroll
        for (int c = 0; c < RC; ++c) acc[c] = 0.f;
        if (lv >= 2) {
            float l[3][N];
            const float p3[3] = {x, y, z};
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                float chi, clo;
                center_pair(geo.lo[d], compact3(key >> d), X.h[lv], chi, clo);
                lagrange_t<N>(cc, local_coord(p3[d], chi, clo, X.inv_h[lv]), l[d]);
            }
#pragma unroll
            for (int c = 0; c < RC; ++c)
                if (c < nr) acc[c] = l2p_sum<N>(X.F[lv] + (int64_t(lcell[q]) * r + c0 + c) * mp, l);
        }
        const float xc = x * cs, yc = y * cs, zc = z * cs;
        for (int w = w0; w < w1; ++w) {
            const int la = wlev[w], a = wcell[w];
            const uint64_t ka = X.keys[la][a];
            const float *M = X.M[la] + (int64_t(a) * r + c0) * mp;
            __syncthreads();                     // previous W cell consumed
            for (int k = lane; k < m; k += 64) {
                float t[3];
                node_coords<N>(cc, geo.lo, ka, X.h[la], cs, k, t);
                nd[k] = make_float4(t[0], t[1], t[2], 0.f);
#pragma unroll
                for (int c = 0; c < RC; ++c) ms[k][c] = c < nr ? M[int64_t(c) * mp + k] : 0.f;
            }
            __syncthreads();
            for (int k = 0; k < m; ++k) {
                const float4 v = nd[k];
                const float kv = kernel_eval<KID>(xc - v.x, yc - v.y, zc - v.z);
#pragma unroll
                for (int c = 0; c < RC; ++c) acc[c] += kv * ms[k][c];
            }
        }
        if (valid) {
            float *out = phi + int64_t(perm[i]) * r + c0;
#pragma unroll
            for (int c = 0; c < RC; ++c)
                if (c < nr) out[c] += acc[c];
        }
    }
}

// The same far field as a product on FP32 MFMA, for blocks of 16 right-hand
// sides: phi[targets][c] += A B with, for M2P over a W cell, A[t][node] =
// K(x_t, y*_node) (lane i + 16 k evaluates target i, node 4 s + k itself into
// its A operand, as the near field does) and B[node][c] the cell's
// coefficients; for L2P, A[t][node] the Lagrange product of the leaf's own
// cell at x_t and B its local expansion.  One wave per (leaf, 16 columns),
// targets in chunks of 64 (four 16-row blocks); a cell's node coordinates
// and 16 columns of coefficients are staged in LDS (nodes padded to a
// multiple of 4 with zero coefficients).
template <int N, int KID>
__global__ void __launch_bounds__(64)
k_leaf_far_mfma(const int32_t *lpb, const int32_t *lpe, const uint64_t *lkey, const int32_t *llev,
                const int32_t *lcell, const int32_t *woff, const int32_t *wlev, const int32_t *wcell,
                LevelExp X, const float *xs, const float *ys, const float *zs, const int32_t *perm,
                Geo geo, ChebConst cc, float cs, int r, int mp, float *phi) {
    constexpr int m = N * N * N, MK = (m + 3) / 4 * 4;
    __shared__ float4 nd[MK];             // node coordinates (kernel units) of the staged cell
    __shared__ float cf[MK][16];          // its coefficients, 16 columns
    __shared__ float Ls[64][3 * N];       // Lagrange values of the chunk's targets
    const int lane = threadIdx.x, row = lane & 15, kq = lane >> 4;
    const int q = blockIdx.x, c0 = blockIdx.y * 16;
    const int nr = min(16, r - c0);
    const int lv = llev[q], b = lpb[q], e = lpe[q];
    const uint64_t key = lkey[q];
    const int w0 = woff[q], w1 = woff[q + 1];
    // stage cell coefficients C[cell][c0 + c][node] (zero past m and past r)
    auto stage_coef = [&](const float *C) {
        for (int g = lane; g < MK * 16; g += 64) {
            const int k = g >> 4, c = g & 15;
            cf[k][c] = (k < m && c < nr) ? C[int64_t(c) * mp + k] : 0.f;
        }
    };
    for (int p0 = b; p0 < e; p0 += 64) {
        float tx[4], ty[4], tz[4];
#pragma unroll
        for (int rb = 0; rb < 4; ++rb) {
            const int ti = p0 + 16 * rb + row;
            const int tc = ti < e ? ti : b;          // rows past the leaf repeat a target; not written
            tx[rb] = xs[tc] * cs;
            ty[rb] = ys[tc] * cs;
            tz[rb] = zs[tc] * cs;
        }
        v4f acc[4];
#pragma unroll
        for (int rb = 0; rb < 4; ++rb) acc[rb] = v4f{0.f, 0.f, 0.f, 0.f};
        if (lv >= 2) {                               // L2P from the leaf's own local expansion
            __syncthreads();                         // LDS of the previous chunk consumed
            {
                const int ti = p0 + lane < e ? p0 + lane : b;
                const float p3[3] = {xs[ti], ys[ti], zs[ti]};
#pragma unroll
                for (int d = 0; d < 3; ++d) {
                    float chi, clo, l[N];
                    center_pair(geo.lo[d], compact3(key >> d), X.h[lv], chi, clo);
                    lagrange_t<N>(cc, local_coord(p3[d], chi, clo, X.inv_h[lv]), l);
#pragma unroll
                    for (int k = 0; k < N; ++k) Ls[lane][d * N + k] = l[k];
                }
            }
            stage_coef(X.F[lv] + (int64_t(lcell[q]) * r + c0) * mp);
            __syncthreads();
            for (int s0 = 0; s0 < MK; s0 += 4) {
                const int node = s0 + kq, nn = node < m ? node : 0;
                const int i1 = nn % N, i2 = (nn / N) % N, i3 = nn / (N * N);
                const float bv = cf[node][row];
#pragma unroll
                for (int rb = 0; rb < 4; ++rb) {
                    const float *L3 = Ls[16 * rb + row];
                    const float av = L3[i1] * L3[N + i2] * L3[2 * N + i3];
                    acc[rb] = __builtin_amdgcn_mfma_f32_16x16x4f32(av, bv, acc[rb], 0, 0, 0);
                }
            }
        }
        for (int w = w0; w < w1; ++w) {             // M2P over the W list
            const int la = wlev[w], a = wcell[w];
            const uint64_t ka = X.keys[la][a];
            __syncthreads();                         // previous cell consumed
            for (int k = lane; k < MK; k += 64) {
                float t[3];
                node_coords<N>(cc, geo.lo, ka, X.h[la], cs, k < m ? k : 0, t);
                nd[k] = make_float4(t[0], t[1], t[2], 0.f);
            }
            stage_coef(X.M[la] + (int64_t(a) * r + c0) * mp);
            __syncthreads();
            for (int s0 = 0; s0 < MK; s0 += 4) {
                const int node = s0 + kq;
                const float4 v = nd[node];
                const float bv = cf[node][row];
#pragma unroll
                for (int rb = 0; rb < 4; ++rb) {
                    const float kv = kernel_eval<KID>(tx[rb] - v.x, ty[rb] - v.y, tz[rb] - v.z);
                    acc[rb] = __builtin_amdgcn_mfma_f32_16x16x4f32(kv, bv, acc[rb], 0, 0, 0);
                }
            }
        }
        // D[i][j] sits in lane j + 16 (i / 4), register i % 4
#pragma unroll
        for (int rb = 0; rb < 4; ++rb)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int ti = p0 + 16 * rb + 4 * kq + v;
                if (ti < e && row < nr) phi[int64_t(perm[ti]) * r + c0 + row] += acc[rb][v];
            }
    }
}

// pleaf[i] = leaf holding point i (tree order)
__global__ void __launch_bounds__(kThreads)
k_point_leaf(const int32_t *pb, const int32_t *pe, int nleaf, int32_t *pleaf) {
    const int a = blockIdx.x * kThreads + threadIdx.x;
    if (a >= nleaf) return;
    for (int i = pb[a]; i < pe[a]; ++i) pleaf[i] = a;
}

inline int grid(int64_t n) { return int(ceil_div(n, kThreads)); }

}  // namespace

// -------------------------------------------------------------- plan ----
constexpr int kTimingRing = 64;
constexpr int kP2PMfmaMinR = 4;         // r from which the near field runs on MFMA by default

struct MaskArgs {
    const int32_t *itab[kMaxLevels];
    const int32_t *oct_cells[kMaxLevels];
};

// masks[tile] bit j = some target of the tile has a source in slot j
__global__ void __launch_bounds__(kThreads) k_tile_masks(const int32_t *tiles, MaskArgs a, uint32_t *masks) {
    __shared__ uint32_t words[kMaskWords];
    const int4 tile = reinterpret_cast<const int4 *>(tiles)[blockIdx.x];
    if (threadIdx.x < kMaskWords) words[threadIdx.x] = 0u;
    __syncthreads();
    const int j = threadIdx.x;
    if (j < kSlots) {
        const int32_t *itab = a.itab[tile.x];
        const int32_t *cells = a.oct_cells[tile.x] + tile.z;
        bool any = false;
        for (int c = 0; c < tile.w && !any; ++c) any = itab[int64_t(cells[c]) * kSlots + j] >= 0;
        if (any) atomicOr(&words[j >> 5], 1u << (j & 31));
    }
    __syncthreads();
    if (threadIdx.x < kMaskWords) masks[int64_t(blockIdx.x) * kMaskWords + threadIdx.x] = words[threadIdx.x];
}

struct Plan {
    const bbfmm_tree *tree = nullptr;
    const bbfmm_ops *ops = nullptr;
    int64_t r = 0;
    int rc_m2l = 1, tpt = 64;           // M2L column tile: tpt targets x rc_m2l rhs
    int nsplit = 1;                     // M2L slot split (partial F^ summed in decompression)
    int rc_p2p = 1;
    bool p2p_mfma = false;              // near field + L2P on MFMA (k_p2p_mfma)
    int ncb_p2p = 1;                    // its 16-column blocks per wave
    int mfma_off[5] = {0};              // its work items with 1..4 row blocks: [off[i], off[i+1])
    // overlapped schedule: the near field on a side stream while the far
    // field runs on the caller's stream, then L2P adds the far field
    bool overlap = false;
    int p2p_waves = 0;                  // per-lane near field: workgroups launched (0 = one per item)
    int m2l_occupancy = 0;              // M2L workgroups per CU (0 = as many as fit)
    int m2l_layout = 1;                 // FP32 M2L waves: 1 = 16 rows x 64 columns, 2 = 32 x 32
    size_t m2l_pad_lds = 0;             // unused dynamic LDS that enforces m2l_occupancy
    hipStream_t side = nullptr;
    hipEvent_t fork = nullptr, join = nullptr;
    DBuf<int32_t> pleaf;                // point -> leaf (tree order), for k_l2p
    DBuf<float> sig_s;                  // sigma in tree order, [N][ld_s]
    int ld_s = 1;                       // r, or whole MFMA column blocks (zero padded)
    DBuf<float> M[kMaxLevels], Mh[kMaxLevels], Fh[kMaxLevels], F[kMaxLevels];
    DBuf<uint16_t> Mh16[kMaxLevels], Ml16[kMaxLevels];   // 16-bit M2L operand formats
    DBuf<float> Msinv[kMaxLevels];                       // fp16 block scales
    DBuf<float2> Mc[kMaxLevels], Fc[kMaxLevels];         // FFT M2L: spectra of M and F
    FftBlocks fblk[kMaxLevels];                          // FFT M2L by spatial blocks
    bool fft_blocked = false;
    DBuf<int32_t> tiles;                // all M2L tiles of all levels
    DBuf<uint32_t> masks;               // per tile: slots in which some target has a source
    int ntiles = 0, max_kp = 0;
    int tile_off[kMaxLevels + 1] = {0};  // first tile of each level (levels >= 2)
    // per-level M2L schedule: the upward chain on `up`, one event per level
    bool m2l_early = false;
    bool m2l_block = false;             // 16-bit M2L by parent blocks (k_m2l_blk), no slot split
    bool m2l_xsplit = false;            // tile M2L: slot splits pinned to XCDs
    bool leaf_fused = false;            // P2M + compression + M2M of the leaf level fused
    bool p2p_pack = false;              // per-lane near field with packed targets (k_p2p_pack)
    bool m2l_w32 = false;               // block M2L on 32x32x16 MFMAs (r-tile >= 32)
    int m2l_cb = 4;                     // its 16-column blocks per workgroup (r-tile / 16)
    hipStream_t up = nullptr;
    hipEvent_t lev_ev[kMaxLevels] = {};
    DBuf<int32_t> work;
    int nwork = 0;
    int64_t ws_bytes = 0;
    // stage timing: a ring of event sets, harvested on query
    bool timing = false;
    std::vector<hipEvent_t> events;     // kTimingRing x (BBFMM_NUM_STAGES + 1)
    int ring_head = 0, ring_pending = 0;
    double stage_ms[BBFMM_NUM_STAGES] = {0};
    int64_t timed_execs = 0;
    // graph replay: the launch sequence captured once per (sigma, phi) pair
    bool graph_on = false;
    hipStream_t cap_stream = nullptr;
    hipGraphExec_t gexec = nullptr;
    const float *g_sigma = nullptr;
    float *g_phi = nullptr;
    // ordering of the plan's products: `done` is recorded after the set-up
    // and after every product on the stream it ran on (`last`); a product on
    // another stream first waits for it, and the destructor waits for it
    bool transient = false;             // one synchronous product: no events, no side stream
    hipEvent_t done = nullptr;
    bool issued = false;
    hipStream_t last = nullptr;
    std::vector<int32_t> h_tiles, h_work;   // host sources of the set-up uploads
    hipStream_t setup = nullptr;        // where the set-up work was enqueued
    Plan() { ++counters().plans; }
    ~Plan() {
        // a plan whose set-up failed (or a transient one) may still have
        // uploads from h_tiles / h_work and mask kernels in flight
        if (!issued) (void)hipStreamSynchronize(setup);
        if (issued) {
            if (hipEventQuery(done) == hipErrorNotReady) ++counters().plans_freed_in_flight;
            (void)hipEventSynchronize(done);
        }
        destroy_event(fork);
        destroy_event(join);
        release_side_stream(side);
        for (hipEvent_t e : lev_ev) destroy_event(e);
        release_side_stream(up);
        for (hipEvent_t e : events) destroy_event(e);
        if (gexec) (void)hipGraphExecDestroy(gexec);
        destroy_stream(cap_stream);
        destroy_event(done);
        --counters().plans;
    }
};

Plan *plan_create_impl(const bbfmm_tree *t, const bbfmm_ops *o, int64_t r,
                       const bbfmm_plan_options *opt, hipStream_t setup, bool transient) {
    bbfmm_plan_options op{};
    if (opt) op = *opt;
    BB_REQUIRE(op.m2l_split >= 0 && op.m2l_split <= 8, "m2l_split must be in [0, 8]");
    BB_REQUIRE(op.m2l_min_waves >= 0 && op.m2l_min_waves <= 16, "m2l_min_waves must be in [0, 16]");
    BB_REQUIRE(op.p2p_max_split >= 0 && op.p2p_max_split <= 64 &&
                   (op.p2p_max_split & (op.p2p_max_split - 1)) == 0,
               "p2p_max_split must be 0 or a power of two <= 64");
    BB_REQUIRE(op.p2p_mfma >= 0 && op.p2p_mfma <= 2, "p2p_mfma must be 0, 1 or 2");
    BB_REQUIRE(op.overlap >= 0 && op.overlap <= 2, "overlap must be 0, 1 or 2");
    BB_REQUIRE(op.p2p_waves >= 0, "p2p_waves must be >= 0");
    BB_REQUIRE(op.m2l_occupancy >= 0 && op.m2l_occupancy <= 4, "m2l_occupancy must be in [0, 4]");
    BB_REQUIRE(op.m2l_layout >= 0 && op.m2l_layout <= 2, "m2l_layout must be 0, 1 or 2");
    BB_REQUIRE(op.m2l_schedule >= 0 && op.m2l_schedule <= 2, "m2l_schedule must be 0, 1 or 2");
    BB_REQUIRE(op.m2l_block >= 0 && op.m2l_block <= 2, "m2l_block must be 0, 1 or 2");
    BB_REQUIRE(op.m2l_rtile == 0 || op.m2l_rtile == 16 || op.m2l_rtile == 32 || op.m2l_rtile == 64,
               "m2l_rtile must be 0, 16, 32 or 64");
    BB_REQUIRE(op.m2l_xcd >= 0 && op.m2l_xcd <= 2, "m2l_xcd must be 0, 1 or 2");
    BB_REQUIRE(op.leaf_fused >= 0 && op.leaf_fused <= 2, "leaf_fused must be 0, 1 or 2");
    BB_REQUIRE(op.p2p_pack >= 0 && op.p2p_pack <= 2, "p2p_pack must be 0, 1 or 2");
    BB_REQUIRE(op.m2l_mfma >= 0 && op.m2l_mfma <= 2, "m2l_mfma must be 0, 1 or 2");
    BB_REQUIRE(t != nullptr && o != nullptr, "tree or ops is NULL");
    BB_REQUIRE(o->tree == t, "operators were built for another tree");
    BB_REQUIRE(r >= 1 && r <= 4096, "r must be in [1, 4096]");
    // the near field's launch lists index the leaf table through the host copies
    BB_INTERNAL(t->leaf_pb_h.size() == size_t(t->leaves().C) &&
                    t->leaf_te_h.size() == size_t(t->leaves().C),
                "leaf ranges do not match the tree's leaves");
    std::unique_ptr<Plan> p(new Plan());
    p->tree = t;
    p->ops = o;
    p->r = r;
    p->transient = transient;
    p->setup = setup;
    const int L = t->leaf_level();
    const int mp = o->mp;
    p->rc_m2l = int(std::min<int64_t>(r, kM2LCols));
    p->tpt = kM2LCols / p->rc_m2l;
    // right-hand sides per per-lane near-field launch column (at most 32: with
    // 64 accumulators per lane the kernel would spill to scratch memory)
    p->rc_p2p = 1;
    while (p->rc_p2p < r && p->rc_p2p < 32) p->rc_p2p *= 2;
    p->p2p_mfma = op.p2p_mfma == 0 ? r >= kP2PMfmaMinR : op.p2p_mfma == 2;
    p->ncb_p2p = r <= 16 ? 1 : (r <= 32 ? 2 : 4);
    p->ld_s = p->p2p_mfma ? int(16 * p->ncb_p2p * ceil_div(r, 16 * p->ncb_p2p)) : int(r);
    p->sig_s.alloc(t->n * p->ld_s);
    int64_t ws = p->sig_s.bytes();
    // the fused leaf pass needs a parent level with expansions (L >= 3)
    // (off by default: on the batched workloads the separate kernels are
    // faster; the autotuner measures both)
    p->leaf_fused = !t->adaptive && L >= 3 && o->precision != BBFMM_M2L_FFT && op.leaf_fused == 2;
    // FFT M2L of a level-uniform tree: by spatial blocks unless asked per cell
    p->fft_blocked = o->precision == BBFMM_M2L_FFT && !t->adaptive && op.m2l_block != 1;
    std::vector<int32_t> tl;
    for (int lvl = 2; lvl <= L; ++lvl) {
        const int64_t C = t->lv[lvl].C;
        const int kp = o->lv[lvl].set->kp;
        p->max_kp = std::max(p->max_kp, kp);
        if (!(p->leaf_fused && lvl == L)) p->M[lvl].alloc(C * r * mp);   // fused: leaf M stays on chip
        p->F[lvl].alloc(C * r * mp);
        if (o->precision == BBFMM_M2L_FFT) {
            const int64_t Q = fft_freqs(o->n);
            p->Mc[lvl].alloc(C * r * Q);
            p->Fc[lvl].alloc(C * r * Q);
            ws += p->Mc[lvl].bytes() + p->Fc[lvl].bytes() + p->M[lvl].bytes() + p->F[lvl].bytes();
            if (p->fft_blocked) {
                fft_build_blocks(t->lv[lvl].keys.p, int32_t(C), lvl, p->fblk[lvl], setup);
                ws += p->fblk[lvl].tgt.bytes() + p->fblk[lvl].halo.bytes() + p->fblk[lvl].slots.bytes();
            }
            continue;            // no compressed operands, no M2L tiles
        } else if (o->precision == BBFMM_M2L_FP32) {
            // one zero cell past the last: the M2L's missing sources read it
            p->Mh[lvl].alloc((C + 1) * r * kp);
            BB_HIP(hipMemsetAsync(p->Mh[lvl].p + C * r * kp, 0, size_t(r) * kp * sizeof(float), setup));
            ws += p->Mh[lvl].bytes();
        } else {
            p->Mh16[lvl].alloc(C * r * kp);
            ws += p->Mh16[lvl].bytes();
            if (o->precision == BBFMM_M2L_BF16X3) {
                p->Ml16[lvl].alloc(C * r * kp);
                ws += p->Ml16[lvl].bytes();
            } else {
                p->Msinv[lvl].alloc(C * r * ceil_div(kp, 64));
                ws += p->Msinv[lvl].bytes();
            }
        }
        ws += p->M[lvl].bytes() + p->F[lvl].bytes();
        // M2L tiles: runs of up to tpt cells of one octant (grouped by the
        // pattern of slots that hold a source, so that a tile's targets
        // share their visited slots; Morton order within a group),
        // interleaved over the octants run by run, so that consecutive tiles
        // -- which the launch deals to one XCD -- cover one region of space
        // and share their sources in that L2
        p->tile_off[lvl] = int(tl.size() / 4);
        const int *oo = t->lv[lvl].oct_off;
        int nrun = 0;
        for (int oc = 0; oc < 8; ++oc) nrun = std::max(nrun, int(ceil_div(oo[oc + 1] - oo[oc], p->tpt)));
        for (int j = 0; j < nrun; ++j)
            for (int oc = 0; oc < 8; ++oc) {
                const int s = oo[oc] + j * p->tpt;
                if (s >= oo[oc + 1]) continue;
                tl.push_back(lvl);
                tl.push_back(oc);
                tl.push_back(s);
                tl.push_back(std::min(p->tpt, oo[oc + 1] - s));
            }
    }
    p->ntiles = int(tl.size() / 4);
    for (int lvl = std::max(L + 1, 2); lvl <= kMaxLevels; ++lvl) p->tile_off[lvl] = p->ntiles;
    // 16-bit M2L for blocks of right-hand sides: parent blocks by default
    // from 16 columns on
    p->m2l_block = (o->precision == BBFMM_M2L_BF16X3 || o->precision == BBFMM_M2L_FP16_SCALED) &&
                   (op.m2l_block == 0 ? r >= 16 : op.m2l_block == 2);
    // r-tile of the parent-block kernel: 16, 32 or 64 columns per workgroup
    p->m2l_cb = op.m2l_rtile > 0 ? op.m2l_rtile / 16 : (r >= 48 ? 4 : (r > 16 ? 2 : 1));
    // MFMA shape of the parent-block kernel: 32x32x16 needs an r-tile of 32 or 64
    p->m2l_w32 = p->m2l_block && p->m2l_cb >= 2 && op.m2l_mfma == 2;
    // split the slots until the launch has about m2l_min_waves workgroups per CU
    if (p->m2l_block) {
        p->nsplit = 1;                  // each block sums its whole halo
    } else if (op.m2l_split > 0) {
        p->nsplit = op.m2l_split;
    } else {
        const int target = op.m2l_min_waves > 0 ? op.m2l_min_waves : 16;
        const int64_t wgs = int64_t(p->ntiles) * ceil_div(p->max_kp, 64) * ceil_div(r, p->rc_m2l);
        while (p->nsplit < 8 && wgs * p->nsplit < int64_t(target) * 256) p->nsplit *= 2;
    }
    // slot splits pinned to XCDs where the split count divides the 8 XCDs
    p->m2l_xsplit = !p->m2l_block && 8 % p->nsplit == 0 && op.m2l_xcd != 1;
    for (int lvl = 2; lvl <= L && o->precision != BBFMM_M2L_FFT; ++lvl) {
        const int64_t C = t->lv[lvl].C;
        p->Fh[lvl].alloc(int64_t(p->nsplit) * C * r * o->lv[lvl].set->kp);
        ws += p->Fh[lvl].bytes();
    }
    if (p->ntiles) {
        p->h_tiles = std::move(tl);
        p->tiles.alloc(p->h_tiles.size());
        BB_HIP(hipMemcpyAsync(p->tiles.p, p->h_tiles.data(), p->h_tiles.size() * sizeof(int32_t),
                              hipMemcpyHostToDevice, setup));
        p->masks.alloc(int64_t(p->ntiles) * kMaskWords);
        MaskArgs ma{};
        for (int lvl = 2; lvl <= L; ++lvl) {
            ma.itab[lvl] = t->lv[lvl].itab.p;
            ma.oct_cells[lvl] = t->lv[lvl].oct_cells.p;
        }
        k_tile_masks<<<p->ntiles, kThreads, 0, setup>>>(p->tiles.p, ma, p->masks.p);
        BB_LAUNCH_CHECK();
        ws += p->tiles.bytes() + p->masks.bytes();
    }
    // overlapped near field: by default with the per-lane near field (whose
    // VALU work complements the MFMA-bound far field); needs a far field
    p->overlap = !transient && L >= 2 && (op.overlap == 0 ? !p->p2p_mfma : op.overlap == 2);
    // packed per-lane near field: one right-hand side; the far field is
    // then added by its own L2P kernel on either schedule
    p->p2p_pack = !p->p2p_mfma && r == 1 && op.p2p_pack != 1;
    if (p->p2p_mfma) {
        // MFMA near field: one wave per (leaf, up to 64 consecutive
        // targets), grouped by the number of 16-row blocks they need
        const LevelData &leaf = t->leaves();
        const std::vector<int32_t> &hb = t->leaf_pb_h, &he = t->leaf_te_h;   // targets of a leaf
        std::vector<int32_t> &w = p->h_work;
        for (int nrb = 1; nrb <= 4; ++nrb) {
            p->mfma_off[nrb - 1] = int(w.size() / 2);
            for (int a = 0; a < leaf.C; ++a)
                for (int s = hb[a]; s < he[a]; s += 64)
                    if (std::min(4, (he[a] - s + 15) / 16) == nrb) {
                        w.push_back(a);
                        w.push_back(s);
                    }
        }
        p->mfma_off[4] = int(w.size() / 2);
        p->nwork = int(w.size() / 2);
        p->work.alloc(w.size());
        BB_HIP(hipMemcpyAsync(p->work.p, w.data(), w.size() * sizeof(int32_t), hipMemcpyHostToDevice,
                              setup));
    } else if (p->p2p_pack) {
        // packed work items (leaf, first target, S | tpl << 5 | G << 8 |
        // count << 15) for `count` consecutive targets of the leaf: G
        // groups of tpl consecutive targets, S sub-lanes each, G S <= 64;
        // per leaf the (tpl, S) that keeps most lanes busy (largest
        // count S / (64 tpl)); on ties fewer targets per lane, then fewer
        // sub-lanes (measured the faster order).  Leaves of
        // more than 64 targets are cut into ceil(count / 64) near-equal
        // pieces, one wave each, so that dense leaves keep as many waves in
        // flight as one target per lane would.
        const LevelData &leaf = t->leaves();
        const std::vector<int32_t> &hb = t->leaf_pb_h, &he = t->leaf_te_h;
        const int cap = op.p2p_max_split > 0 ? std::min(op.p2p_max_split, 16) : 16;
        std::vector<int32_t> &w = p->h_work;
        for (int a = 0; a < leaf.C; ++a) {
            const int total = he[a] - hb[a];
            const int pieces = (total + 63) / 64;
            for (int q = 0, s0 = hb[a]; q < pieces; ++q) {
                const int cnt = total / pieces + (q < total % pieces ? 1 : 0);
                int best_t = 4, best_s = 1;
                double best = -1.0;
                for (int tpl : {1, 2, 4})
                    for (int S = 1; S <= cap; ++S) {
                        const int G = (cnt + tpl - 1) / tpl;
                        if (G * S > 64) break;
                        const double eff = double(cnt) * S / (64.0 * tpl);
                        if (eff > best + 1e-12) {
                            best = eff;
                            best_t = tpl;
                            best_s = S;
                        }
                    }
                const int G = (cnt + best_t - 1) / best_t;
                w.push_back(a);
                w.push_back(s0);
                w.push_back(best_s | (best_t << 5) | (G << 8) | (cnt << 15));
                s0 += cnt;
            }
        }
        p->nwork = int(w.size() / 3);
        p->work.alloc(w.size());
        BB_HIP(hipMemcpyAsync(p->work.p, w.data(), w.size() * sizeof(int32_t), hipMemcpyHostToDevice,
                              setup));
    } else {
        // per-lane P2P work items (leaf, first target, log2 S): leaves of at
        // most 64 points take one wave with 64 / next_pow2(count) sub-lanes
        // per target
        const LevelData &leaf = t->leaves();
        const std::vector<int32_t> &hb = t->leaf_pb_h, &he = t->leaf_te_h;   // targets of a leaf
        std::vector<int32_t> &w = p->h_work;
        for (int a = 0; a < leaf.C; ++a) {
            const int cnt = he[a] - hb[a];
            int lgT = 0;
            while ((1 << lgT) < std::min(cnt, 64)) ++lgT;
            const int cap = op.p2p_max_split > 0 ? std::min(op.p2p_max_split, 16) : 16;
            while ((64 >> lgT) > cap) ++lgT;   // at most cap sub-lanes per target
            for (int s = hb[a]; s < he[a]; s += (1 << lgT)) {
                w.push_back(a);
                w.push_back(s);
                w.push_back(6 - lgT);
            }
        }
        p->nwork = int(w.size() / 3);
        p->work.alloc(w.size());
        BB_HIP(hipMemcpyAsync(p->work.p, w.data(), w.size() * sizeof(int32_t), hipMemcpyHostToDevice,
                              setup));
    }
    p->p2p_waves = op.p2p_waves;
    p->m2l_occupancy = op.m2l_occupancy;
    p->m2l_layout = op.m2l_layout == 2 ? 2 : 1;
    if (op.m2l_occupancy > 0 && L >= 2) {
        // pad the M2L workgroup's LDS so that at most m2l_occupancy fit on a
        // CU (160 KiB of LDS each), leaving registers to a concurrent kernel
        hipFuncAttributes fa{};
        if (o->precision == BBFMM_M2L_FP32)
            BB_HIP(hipFuncGetAttributes(&fa, op.m2l_layout == 2 ? reinterpret_cast<const void *>(k_m2l<2, false>)
                                                              : reinterpret_cast<const void *>(k_m2l<4, false>)));
        else if (o->precision == BBFMM_M2L_BF16X3)
            BB_HIP(hipFuncGetAttributes(&fa, reinterpret_cast<const void *>(k_m2l_lp<BBFMM_M2L_BF16X3>)));
        else
            BB_HIP(hipFuncGetAttributes(&fa, reinterpret_cast<const void *>(k_m2l_lp<BBFMM_M2L_FP16_SCALED>)));
        const size_t per_wg = size_t(160 * 1024) / size_t(op.m2l_occupancy) - 512;
        p->m2l_pad_lds = per_wg > fa.sharedSizeBytes ? per_wg - fa.sharedSizeBytes : 0;
    }
    // a separate L2P kernel (k_l2p) after the near field: on the overlapped
    // schedule and with the packed near field (adaptive trees: k_leaf_far)
    if (!t->adaptive && L >= 2 && (p->overlap || p->p2p_pack)) {
        const LevelData &leaf = t->lv[L];
        p->pleaf.alloc(t->n);
        ws += p->pleaf.bytes();
        k_point_leaf<<<grid(leaf.C), kThreads, 0, setup>>>(leaf.pb.p, leaf.pe.p, leaf.C,
                                                           p->pleaf.p);
        BB_LAUNCH_CHECK();
    }
    if (p->overlap) {
        p->side = acquire_side_stream();
        p->fork = make_event(hipEventDisableTiming);
        p->join = make_event(hipEventDisableTiming);
    }
    // per-level M2L schedule (default on with at least two M2L levels)
    p->m2l_early = !transient && L >= 3 && o->precision != BBFMM_M2L_FFT &&
                   (op.m2l_schedule == 0 || op.m2l_schedule == 2);
    if (p->m2l_early) {
        p->up = acquire_side_stream();
        for (int lvl = 2; lvl <= L; ++lvl) p->lev_ev[lvl] = make_event(hipEventDisableTiming);
    }
    p->ws_bytes = ws;
    if (!transient) {
        p->done = make_event(hipEventDisableTiming);
        BB_HIP(hipEventRecord(p->done, setup));
        p->issued = true;
        p->last = setup;
    }
    return p.release();
}

int64_t plan_workspace_bytes(const Plan *p) { return p->ws_bytes; }

void plan_resolved_options(const Plan *p, bbfmm_plan_options *out) {
    out->m2l_split = p->nsplit;
    out->p2p_mfma = p->p2p_mfma ? 2 : 1;
    out->overlap = p->overlap ? 2 : 1;
    out->p2p_waves = p->p2p_waves;
    out->m2l_occupancy = p->m2l_occupancy;
    out->m2l_layout = p->m2l_layout;
    out->m2l_schedule = p->m2l_early ? 2 : 1;
    out->m2l_block = (p->m2l_block || p->fft_blocked) ? 2 : 1;
    out->m2l_rtile = 16 * p->m2l_cb;
    out->m2l_xcd = p->m2l_xsplit ? 2 : 1;
    out->leaf_fused = p->leaf_fused ? 2 : 1;
    out->p2p_pack = p->p2p_pack ? 2 : 1;
    out->m2l_mfma = p->m2l_w32 ? 2 : 1;
    if (out->p2p_max_split == 0) out->p2p_max_split = 16;   // the per-lane kernel's default cap
}
void plan_destroy(Plan *p) { delete p; }

namespace {

// per execution: the stage boundaries on the caller's stream, then (the
// overlapped schedule) P2P start / end on the side stream and the point
// after the join where L2P starts, then (the per-level M2L schedule) the
// start and end of the upward chain on its own stream
constexpr int kEv = BBFMM_NUM_STAGES + 1 + 5;
constexpr int kEvSideBeg = BBFMM_NUM_STAGES + 1, kEvSideEnd = kEvSideBeg + 1, kEvJoined = kEvSideBeg + 2;
constexpr int kEvUpBeg = kEvSideBeg + 3, kEvUpEnd = kEvSideBeg + 4;

// fold the oldest pending execution's stage times into the totals
void harvest_one(Plan &p) {
    const int slot = (p.ring_head - p.ring_pending + kTimingRing) % kTimingRing;
    hipEvent_t *ev = &p.events[size_t(slot) * kEv];
    BB_HIP(hipEventSynchronize(ev[BBFMM_NUM_STAGES]));
    for (int st = 0; st < BBFMM_NUM_STAGES; ++st) {
        float ms = 0.f;
        if (p.m2l_early && st == BBFMM_STAGE_M2M) {
            BB_HIP(hipEventElapsedTime(&ms, ev[kEvUpBeg], ev[kEvUpEnd]));
        } else if (p.m2l_early && st == BBFMM_STAGE_M2L) {
            BB_HIP(hipEventElapsedTime(&ms, ev[BBFMM_STAGE_M2L], ev[BBFMM_STAGE_DOWN]));
        } else if (p.overlap && st == BBFMM_STAGE_P2P) {
            // near field on the side stream + L2P after the join
            float l2p = 0.f;
            BB_HIP(hipEventElapsedTime(&ms, ev[kEvSideBeg], ev[kEvSideEnd]));
            BB_HIP(hipEventElapsedTime(&l2p, ev[kEvJoined], ev[BBFMM_NUM_STAGES]));
            ms += l2p;
        } else {
            BB_HIP(hipEventElapsedTime(&ms, ev[st], ev[st + 1]));
        }
        p.stage_ms[st] += ms;
    }
    --p.ring_pending;
    ++p.timed_execs;
}

template <int KID>
void launch_p2p(const Plan &p, const float *FL, const Geo &geo, float *phi, hipStream_t s) {
    const bbfmm_tree &t = *p.tree;
    const LevelData &leaf = t.leaves();
    const double a = t.params.kernel_param;
    const float cs = coord_scale(t.params.kernel_id, a);
    if (p.p2p_mfma) {
        for (int nrb = 1; nrb <= 4; ++nrb) {
            const int w0 = p.mfma_off[nrb - 1], nw = p.mfma_off[nrb] - w0;
            if (nw == 0) continue;
            dim3 g(unsigned(nw), unsigned(ceil_div(p.r, 16 * p.ncb_p2p)));
            const int32_t *wk = p.work.p + 2 * int64_t(w0);
#define BB_P2PM(NCB, NRB)                                                                     \
            k_p2p_mfma<KID, NCB, NRB><<<g, 64, 0, s>>>(t.xs.p, t.ys.p, t.zs.p, t.src_begin(),    \
                leaf.pe.p, t.tgt_end(), t.nbr_off.p, t.nbr_idx.p, leaf.keys.p, t.perm.p, wk,     \
                p.sig_s.p, p.ld_s, int(p.r), cs, FL, p.ops->mp, geo, p.ops->cheb, phi)
#define BB_P2PM_R(NCB)                                                                        \
            switch (nrb) {                                                                    \
            case 1: BB_P2PM(NCB, 1); break;                                                   \
            case 2: BB_P2PM(NCB, 2); break;                                                   \
            case 3: BB_P2PM(NCB, 3); break;                                                   \
            default: BB_P2PM(NCB, 4); break;                                                  \
            }
            switch (p.ncb_p2p) {
            case 1: BB_P2PM_R(1); break;
            case 2: BB_P2PM_R(2); break;
            default: BB_P2PM_R(4); break;
            }
#undef BB_P2PM_R
#undef BB_P2PM
            BB_LAUNCH_CHECK();
        }
        return;
    }
    const int nwg = p.p2p_waves > 0 ? std::min(p.p2p_waves, p.nwork) : p.nwork;
    if (p.p2p_pack) {
        BB_INTERNAL(FL == nullptr && p.r == 1, "the packed near field takes one column and no L2P");
        if (nwg == 0) return;
        k_p2p_pack<KID><<<nwg, 64, 0, s>>>(t.xs.p, t.ys.p, t.zs.p, t.src_begin(), leaf.pe.p,
                                           t.tgt_end(), t.nbr_off.p, t.nbr_idx.p, t.perm.p,
                                           p.work.p, p.nwork, p.sig_s.p, p.ld_s, cs, phi);
        BB_LAUNCH_CHECK();
        return;
    }
    dim3 g(unsigned(nwg), unsigned(ceil_div(p.r, p.rc_p2p)));
#define BB_P2P(RCV)                                                                          \
    k_p2p<KID, RCV><<<g, 64, 0, s>>>(t.xs.p, t.ys.p, t.zs.p, t.src_begin(), leaf.pe.p,        \
                                     t.tgt_end(), t.nbr_off.p, t.nbr_idx.p, leaf.keys.p,      \
                                     t.perm.p, p.work.p, p.nwork, p.sig_s.p, int(p.r), cs,   \
                                     FL, p.ops->mp, geo, p.ops->cheb, phi)
    switch (p.rc_p2p) {
    case 1: BB_P2P(1); break;
    case 2: BB_P2P(2); break;
    case 4: BB_P2P(4); break;
    case 8: BB_P2P(8); break;
    case 16: BB_P2P(16); break;
    default: BB_P2P(32); break;
    }
#undef BB_P2P
    BB_LAUNCH_CHECK();
}

// L2P + M2P at every leaf of a level-adaptive tree (k_leaf_far)
template <int KID>
void launch_leaf_far(const Plan &p, const Geo &geo, float *phi, hipStream_t s) {
    const bbfmm_tree &t = *p.tree;
    const LevelData &fl = t.leaves();
    if (fl.C == 0) return;
    LevelExp X{};
    for (int l = 0; l < t.depth; ++l) {
        X.keys[l] = t.lv[l].keys.p;
        X.h[l] = float(t.half_width(l));
        X.inv_h[l] = 1.0f / X.h[l];
        if (l >= 2) {
            X.F[l] = p.F[l].p;
            X.M[l] = p.M[l].p;
        }
    }
    const float cs = coord_scale(t.params.kernel_id, t.params.kernel_param);
    const int mp = p.ops->mp, r = int(p.r);
    if (p.p2p_mfma) {                       // as a product on MFMA, 16 columns per wave
        dim3 g(unsigned(fl.C), unsigned(ceil_div(r, 16)));
#define BB_LFM(NN) case NN: k_leaf_far_mfma<NN, KID><<<g, 64, 0, s>>>(fl.pb.p, fl.pe.p, fl.keys.p, \
        t.fl_level.p, t.fl_cell.p, t.w_off.p, t.w_level.p, t.w_cell.p, X, t.xs.p, t.ys.p, t.zs.p, \
        t.perm.p, geo, p.ops->cheb, cs, r, mp, phi); break;
        switch (p.ops->n) {
        BB_LFM(2) BB_LFM(3) BB_LFM(4) BB_LFM(5) BB_LFM(6) BB_LFM(7) BB_LFM(8)
        }
#undef BB_LFM
        BB_LAUNCH_CHECK();
        return;
    }
    // columns per wave: one, or blocks of 16 (each kernel value serves them all)
    const int rc = r == 1 ? 1 : 16;
    dim3 g(unsigned(fl.C), unsigned(ceil_div(r, rc)));
#define BB_LF1(NN, RCC) k_leaf_far<NN, KID, RCC><<<g, 64, 0, s>>>(fl.pb.p, fl.pe.p, fl.keys.p,     \
        t.fl_level.p, t.fl_cell.p, t.w_off.p, t.w_level.p, t.w_cell.p, X, t.xs.p, t.ys.p, t.zs.p, \
        t.perm.p, geo, p.ops->cheb, cs, r, mp, phi)
#define BB_LF(NN) case NN: if (rc == 1) BB_LF1(NN, 1); else BB_LF1(NN, 16); break;
    switch (p.ops->n) {
    BB_LF(2) BB_LF(3) BB_LF(4) BB_LF(5) BB_LF(6) BB_LF(7) BB_LF(8)
    }
#undef BB_LF
#undef BB_LF1
    BB_LAUNCH_CHECK();
}

void leaf_far(const Plan &p, const Geo &geo, float *phi, hipStream_t s) {
    switch (p.tree->params.kernel_id) {
    case BBFMM_K_INV_R: launch_leaf_far<BBFMM_K_INV_R>(p, geo, phi, s); break;
    case BBFMM_K_EXP: launch_leaf_far<BBFMM_K_EXP>(p, geo, phi, s); break;
    case BBFMM_K_GAUSS: launch_leaf_far<BBFMM_K_GAUSS>(p, geo, phi, s); break;
    case BBFMM_K_DIPOLE_X: launch_leaf_far<BBFMM_K_DIPOLE_X>(p, geo, phi, s); break;
    default: launch_leaf_far<BBFMM_K_POLY_TEST>(p, geo, phi, s); break;
    }
}

}  // namespace

void plan_set_timing(Plan *p, bool on) {
    BB_REQUIRE(p != nullptr, "plan is NULL");
    if (on && p->events.empty()) {
        p->events.reserve(size_t(kTimingRing) * kEv);
        for (int i = 0; i < kTimingRing * kEv; ++i) p->events.push_back(make_event(hipEventDefault));
    }
    if (!on)
        while (p->ring_pending > 0) harvest_one(*p);
    p->timing = on;
}

void plan_stage_times(Plan *p, double *ms, int64_t *execs, bool reset) {
    BB_REQUIRE(p != nullptr, "plan is NULL");
    while (p->ring_pending > 0) harvest_one(*p);
    if (ms)
        for (int st = 0; st < BBFMM_NUM_STAGES; ++st) ms[st] = p->stage_ms[st];
    if (execs) *execs = p->timed_execs;
    if (reset) {
        for (double &v : p->stage_ms) v = 0.0;
        p->timed_execs = 0;
    }
}

namespace {
void enqueue_matvec(Plan &p, const float *sigma, float *phi, hipStream_t s, bool timing);
}

void plan_set_graph(Plan *p, bool on) {
    BB_REQUIRE(p != nullptr, "plan is NULL");
    BB_REQUIRE(!(on && p->transient), "a transient plan has no graph");
    if (on && p->cap_stream == nullptr) p->cap_stream = make_stream();
    if (!on && p->gexec) {
        BB_HIP(hipGraphExecDestroy(p->gexec));
        p->gexec = nullptr;
    }
    p->graph_on = on;
}

void plan_execute_impl(Plan *pp, const float *sigma, float *phi, hipStream_t s) {
    BB_REQUIRE(pp != nullptr, "plan is NULL");
    BB_REQUIRE(sigma != nullptr && phi != nullptr, "sigma / phi is NULL");
    Plan &p = *pp;
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    BB_HIP(hipStreamIsCapturing(s, &cap));
    const bool track = !p.transient && cap == hipStreamCaptureStatusNone;
    // the workspace serves one product at a time: wait for the previous one
    // when it ran on another stream
    if (track && p.issued && p.last != s) BB_HIP(hipStreamWaitEvent(s, p.done, 0));
    if (!p.graph_on) {
        enqueue_matvec(p, sigma, phi, s, p.timing);
    } else {
        if (p.gexec == nullptr || sigma != p.g_sigma || phi != p.g_phi) {
            if (p.gexec) {
                BB_HIP(hipGraphExecDestroy(p.gexec));
                p.gexec = nullptr;
            }
            BB_HIP(hipStreamBeginCapture(p.cap_stream, hipStreamCaptureModeThreadLocal));
            hipGraph_t graph = nullptr;
            try {
                enqueue_matvec(p, sigma, phi, p.cap_stream, false);
            } catch (...) {
                (void)hipStreamEndCapture(p.cap_stream, &graph);
                if (graph) (void)hipGraphDestroy(graph);
                throw;
            }
            BB_HIP(hipStreamEndCapture(p.cap_stream, &graph));
            const hipError_t e = hipGraphInstantiate(&p.gexec, graph, nullptr, nullptr, 0);
            (void)hipGraphDestroy(graph);
            BB_HIP(e);
            p.g_sigma = sigma;
            p.g_phi = phi;
        }
        BB_HIP(hipGraphLaunch(p.gexec, s));
    }
    if (track) {
        BB_HIP(hipEventRecord(p.done, s));
        p.issued = true;
        p.last = s;
    }
}

// ------------------------------------------------ bbfmm_matvec cache ----
constexpr size_t kCachedPlans = 4;

struct PlanCache {
    struct Item {
        int64_t r;
        hipStream_t s;
        Plan *plan;
        uint64_t use;
    };
    std::vector<Item> items;
    uint64_t tick = 0;
};

void plan_cache_destroy(PlanCache *c) {
    if (!c) return;
    for (PlanCache::Item &it : c->items) delete it.plan;   // waits for its last product
    delete c;
}

void matvec_cached(bbfmm_ops *o, const float *sigma, int64_t r, float *phi, hipStream_t s) {
    std::lock_guard<std::mutex> lk(o->cache_mu);
    if (o->cache == nullptr) o->cache = new PlanCache();
    PlanCache &c = *o->cache;
    Plan *plan = nullptr;
    for (PlanCache::Item &it : c.items)
        if (it.r == r && it.s == s) {
            it.use = ++c.tick;
            plan = it.plan;
        }
    if (plan == nullptr) {
        MemScope scope(&o->hook, s);
        std::unique_ptr<Plan> fresh(plan_create_impl(o->tree, o, r, nullptr, s));
        if (c.items.size() >= kCachedPlans) {
            size_t victim = 0;
            for (size_t i = 1; i < c.items.size(); ++i)
                if (c.items[i].use < c.items[victim].use) victim = i;
            delete c.items[victim].plan;
            c.items.erase(c.items.begin() + long(victim));
        }
        c.items.push_back(PlanCache::Item{r, s, fresh.get(), ++c.tick});
        plan = fresh.release();
    }
    plan_execute_impl(plan, sigma, phi, s);
}

namespace {
void enqueue_matvec(Plan &p, const float *sigma, float *phi, hipStream_t s, bool timing) {
    const bbfmm_tree &t = *p.tree;
    const bbfmm_ops &o = *p.ops;
    const int L = t.leaf_level();
    const int r = int(p.r);
    Geo geo;
    for (int d = 0; d < 3; ++d) geo.lo[d] = t.lo[d];
    geo.h = float(t.half_width(L));
    geo.inv_h = 1.0f / geo.h;

    hipEvent_t *ev = nullptr;
    if (timing) {
        if (p.ring_pending == kTimingRing) harvest_one(p);
        ev = &p.events[size_t(p.ring_head) * kEv];
        p.ring_head = (p.ring_head + 1) % kTimingRing;
        ++p.ring_pending;
    }
    auto mark = [&](int st) {
        if (ev) BB_HIP(hipEventRecord(ev[st], s));
    };

    mark(BBFMM_STAGE_GATHER);
    k_gather_sigma<<<grid(t.n * p.ld_s), kThreads, 0, s>>>(sigma, t.perm.p, t.n, r, p.ld_s,
                                                           int(t.n_targets), p.sig_s.p);
    BB_LAUNCH_CHECK();
    const float *FL = nullptr;
    const int n = o.n, mp = o.mp;
    auto near_field = [&](const float *fl, hipStream_t st) {
        switch (t.params.kernel_id) {
        case BBFMM_K_INV_R: launch_p2p<BBFMM_K_INV_R>(p, fl, geo, phi, st); break;
        case BBFMM_K_EXP: launch_p2p<BBFMM_K_EXP>(p, fl, geo, phi, st); break;
        case BBFMM_K_GAUSS: launch_p2p<BBFMM_K_GAUSS>(p, fl, geo, phi, st); break;
        case BBFMM_K_DIPOLE_X: launch_p2p<BBFMM_K_DIPOLE_X>(p, fl, geo, phi, st); break;
        default: launch_p2p<BBFMM_K_POLY_TEST>(p, fl, geo, phi, st); break;
        }
    };
    if (p.overlap) {
        // the near field writes phi on the side stream meanwhile
        BB_HIP(hipEventRecord(p.fork, s));
        BB_HIP(hipStreamWaitEvent(p.side, p.fork, 0));
        if (ev) BB_HIP(hipEventRecord(ev[kEvSideBeg], p.side));
        near_field(nullptr, p.side);
        if (ev) BB_HIP(hipEventRecord(ev[kEvSideEnd], p.side));
        BB_HIP(hipEventRecord(p.join, p.side));
    }
    mark(BBFMM_STAGE_P2M);
    if (p.leaf_fused) {
        // P2M, compression and M2M of the leaf level (k_leaf_up)
        const OpSet &set = *o.lv[L].set;
        LeafUpArgs la{};
        la.xs = t.xs.p;
        la.ys = t.ys.p;
        la.zs = t.zs.p;
        la.sb = t.src_begin();
        la.pe = t.lv[L].pe.p;
        la.keys = t.lv[L].keys.p;
        la.pcb = t.lv[L - 1].cb.p;
        la.pce = t.lv[L - 1].ce.p;
        la.sig_s = p.sig_s.p;
        la.ld = p.ld_s;
        la.r = r;
        la.mp = mp;
        la.kp = set.kp;
        la.nchunk = int(ceil_div(set.kp, 64));
        la.VT = set.VT32.p;
        la.Mh = p.Mh[L].p;
        la.Mh16 = p.Mh16[L].p;
        la.Ml16 = p.Ml16[L].p;
        la.Msinv = p.Msinv[L].p;
        la.Mpar = p.M[L - 1].p;
        dim3 g(unsigned(t.lv[L - 1].C), unsigned(ceil_div(r, 16)));
#define BB_LU(NN)                                                                                   \
        case NN:                                                                                    \
            if (o.precision == BBFMM_M2L_FP32)                                                      \
                k_leaf_up<NN, kOutF32><<<g, kThreads, 0, s>>>(la, geo, o.cheb);                     \
            else if (o.precision == BBFMM_M2L_BF16X3)                                               \
                k_leaf_up<NN, kOutBF16X3><<<g, kThreads, 0, s>>>(la, geo, o.cheb);                  \
            else                                                                                    \
                k_leaf_up<NN, kOutF16S><<<g, kThreads, 0, s>>>(la, geo, o.cheb);                    \
            break;
        switch (n) { BB_LU(2) BB_LU(3) BB_LU(4) BB_LU(5) BB_LU(6) BB_LU(7) BB_LU(8) }
#undef BB_LU
        BB_LAUNCH_CHECK();
    } else if (L >= 2 && t.adaptive) {
        // leaves of every level >= 2 (M2M skips them)
        const LevelData &fl = t.leaves();
        for (int lvl = 2; lvl <= L; ++lvl) {
            const LevelData &lv = t.lv[lvl];
            if (lv.nleaf == 0) continue;
            Geo gl = geo;
            gl.h = float(t.half_width(lvl));
            gl.inv_h = 1.0f / gl.h;
            const int32_t *lpb = fl.pb.p + lv.leaf0, *lpe = fl.pe.p + lv.leaf0;
            const uint64_t *lk = fl.keys.p + lv.leaf0;
            const int32_t *rows = t.fl_cell.p + lv.leaf0;
            if (p.p2p_mfma) {
                dim3 g(unsigned(lv.nleaf), unsigned(p.ld_s / (16 * p.ncb_p2p)));
#define BB_P2MM(NN, NCB) k_p2m_mfma<NN, NCB><<<g, kThreads, 0, s>>>(t.xs.p, t.ys.p, t.zs.p, lpb,                     lpe, lk, rows, gl, o.cheb, p.sig_s.p, p.ld_s, r, mp, p.M[lvl].p)
#define BB_P2MN(NN) case NN:                                                                                      if (p.ncb_p2p == 1) BB_P2MM(NN, 1);                                                           else if (p.ncb_p2p == 2) BB_P2MM(NN, 2);                                                      else BB_P2MM(NN, 4);                                                                          break;
                switch (n) {
                    BB_P2MN(2) BB_P2MN(3) BB_P2MN(4) BB_P2MN(5) BB_P2MN(6) BB_P2MN(7) BB_P2MN(8)
                }
#undef BB_P2MN
#undef BB_P2MM
            } else {
                switch (n) {
#define BB_P2M(NN) case NN: k_p2m<NN><<<dim3(unsigned(ceil_div(lv.nleaf, 64 / ((NN) * (NN)))), unsigned(r)),                     64, 0, s>>>(t.xs.p, t.ys.p, t.zs.p, lpb, lpe, lk, rows, lv.nleaf, gl, o.cheb,                          p.sig_s.p, p.ld_s, r, mp, p.M[lvl].p); break;
                BB_P2M(2) BB_P2M(3) BB_P2M(4) BB_P2M(5) BB_P2M(6) BB_P2M(7) BB_P2M(8)
#undef BB_P2M
                }
            }
            BB_LAUNCH_CHECK();
        }
    } else if (L >= 2 && p.p2p_mfma) {
        // blocks of right-hand sides: P2M on MFMA (sigma padded to whole column blocks)
        const LevelData &leaf = t.lv[L];
        dim3 g(leaf.C, unsigned(p.ld_s / (16 * p.ncb_p2p)));
#define BB_P2MM(NN, NCB) k_p2m_mfma<NN, NCB><<<g, kThreads, 0, s>>>(t.xs.p, t.ys.p, t.zs.p, t.src_begin(), \
            leaf.pe.p, leaf.keys.p, nullptr, geo, o.cheb, p.sig_s.p, p.ld_s, r, mp, p.M[L].p)
#define BB_P2MN(NN) case NN:                                                                  \
            if (p.ncb_p2p == 1) BB_P2MM(NN, 1);                                               \
            else if (p.ncb_p2p == 2) BB_P2MM(NN, 2);                                          \
            else BB_P2MM(NN, 4);                                                              \
            break;
        switch (n) {
            BB_P2MN(2) BB_P2MN(3) BB_P2MN(4) BB_P2MN(5) BB_P2MN(6) BB_P2MN(7) BB_P2MN(8)
        }
#undef BB_P2MN
#undef BB_P2MM
        BB_LAUNCH_CHECK();
    } else if (L >= 2) {
        const LevelData &leaf = t.lv[L];
        switch (n) {
#define BB_P2M(NN) case NN: k_p2m<NN><<<dim3(unsigned(ceil_div(leaf.C, 64 / ((NN) * (NN)))), unsigned(r)), \
            64, 0, s>>>(t.xs.p, t.ys.p, t.zs.p, t.src_begin(), leaf.pe.p, leaf.keys.p, nullptr, \
            int(leaf.C), geo, o.cheb, p.sig_s.p, p.ld_s, r, mp, p.M[L].p); break;
        BB_P2M(2) BB_P2M(3) BB_P2M(4) BB_P2M(5) BB_P2M(6) BB_P2M(7) BB_P2M(8)
#undef BB_P2M
        }
        BB_LAUNCH_CHECK();
    }
    auto compress = [&](int lvl, hipStream_t st) {
        if (o.precision == BBFMM_M2L_FFT) {     // the multipoles' spectra instead
            fft_forward(n, p.M[lvl].p, mp, int64_t(t.lv[lvl].C) * r, p.Mc[lvl].p, st);
            return;
        }
        const OpSet &set = *o.lv[lvl].set;
        const int64_t R = int64_t(t.lv[lvl].C) * r;
        const int nchunk = int(ceil_div(set.kp, 64));
        dim3 g(unsigned(ceil_div(R, 64)), unsigned(nchunk));
        if (o.precision == BBFMM_M2L_FP32)
            k_gemm_nt<kOutF32><<<g, kThreads, 0, st>>>(p.M[lvl].p, mp, 1, 0, set.VT32.p, mp,
                                                     p.Mh[lvl].p, set.kp, R, set.kp, mp, 1.f, 0.f,
                                                     nullptr, nullptr, nullptr, 0);
        else if (o.precision == BBFMM_M2L_BF16X3)
            k_gemm_nt<kOutBF16X3><<<g, kThreads, 0, st>>>(p.M[lvl].p, mp, 1, 0, set.VT32.p, mp,
                                                        nullptr, set.kp, R, set.kp, mp, 1.f, 0.f,
                                                        p.Mh16[lvl].p, p.Ml16[lvl].p, nullptr, 0);
        else
            k_gemm_nt<kOutF16S><<<g, kThreads, 0, st>>>(p.M[lvl].p, mp, 1, 0, set.VT32.p, mp,
                                                      nullptr, set.kp, R, set.kp, mp, 1.f, 0.f,
                                                      p.Mh16[lvl].p, nullptr, p.Msinv[lvl].p,
                                                      nchunk);
        BB_LAUNCH_CHECK();
    };
    auto m2m = [&](int lvl, hipStream_t st) {
        const LevelData &lv = t.lv[lvl], &ch = t.lv[lvl + 1];
        switch (n) {
#define BB_M2M(NN) case NN: k_m2m_pen<NN><<<dim3(unsigned(lv.C), unsigned(ceil_div(r, Pencil<NN>::G))), \
            64, 0, st>>>(lv.cb.p, lv.ce.p, ch.keys.p, p.M[lvl + 1].p, o.cheb, r, mp, p.M[lvl].p); break;
        BB_M2M(2) BB_M2M(3) BB_M2M(4) BB_M2M(5) BB_M2M(6) BB_M2M(7) BB_M2M(8)
#undef BB_M2M
        }
        BB_LAUNCH_CHECK();
    };
    // one M2L launch over the tiles of levels lo..hi
    auto m2l = [&](int lo, int hi, hipStream_t st) {
        if (p.m2l_block) {
            for (int lvl = lo; lvl <= hi; ++lvl) {
                const OpSet &set = *o.lv[lvl].set;
                const int kp = set.kp;
                M2LBlockArgs g{p.Mh16[lvl].p, p.Ml16[lvl].p, p.Msinv[lvl].p, p.Fh[lvl].p,
                               o.precision == BBFMM_M2L_BF16X3 ? set.Chi.p : set.C16.p, set.Clo.p,
                               set.Cinv.p, t.lv[lvl].itab.p, t.lv[lvl].keys.p, t.lv[lvl - 1].cb.p,
                               t.lv[lvl - 1].ce.p, t.tables.p + 3 * kNumT + 8 * kSlots, kp, r};
                const int CBv = p.m2l_cb;
                const bool w32 = p.m2l_w32 && CBv >= 2;   // 32x32x16 MFMAs: 32 rows
                const int RBv = (w32 || kp <= 32 || CBv == 4 ||
                                 (CBv == 2 && o.precision == BBFMM_M2L_BF16X3)) ? 2 : 4;
                dim3 gr(unsigned(t.lv[lvl - 1].C), unsigned(ceil_div(kp, 16 * RBv)),
                        unsigned(ceil_div(r, 16 * CBv)));
#define BB_BLK(PR, RBc, CBc, W) k_m2l_blk<PR, RBc, CBc, W><<<gr, kThreads, p.m2l_pad_lds, st>>>(g)
#define BB_BLK_P(PR)                                                                          \
                if (w32 && CBv == 2) BB_BLK(PR, 2, 2, true);                                  \
                else if (w32) BB_BLK(PR, 2, 4, true);                                         \
                else if (RBv == 2 && CBv == 1) BB_BLK(PR, 2, 1, false);                       \
                else if (RBv == 2 && CBv == 2) BB_BLK(PR, 2, 2, false);                       \
                else if (RBv == 2) BB_BLK(PR, 2, 4, false);                                   \
                else if (CBv == 1) BB_BLK(PR, 4, 1, false);                                   \
                else BB_BLK(PR, 4, 2, false);
                if (o.precision == BBFMM_M2L_BF16X3) {
                    BB_BLK_P(BBFMM_M2L_BF16X3)
                } else {
                    BB_BLK_P(BBFMM_M2L_FP16_SCALED)
                }
#undef BB_BLK_P
#undef BB_BLK
                BB_LAUNCH_CHECK();
            }
            return;
        }
        if (o.precision == BBFMM_M2L_FFT) {
            for (int lvl = lo; lvl <= hi; ++lvl)
                if (p.fft_blocked)
                    fft_m2l_blocks(n, p.Mc[lvl].p, o.lv[lvl].set->Ghat.p, p.fblk[lvl], r, p.Fc[lvl].p, st);
                else
                    fft_m2l(n, p.Mc[lvl].p, o.lv[lvl].set->Ghat.p, t.lv[lvl].itab.p, t.lv[lvl].keys.p,
                            t.tables.p + 3 * kNumT, t.lv[lvl].C, r, p.Fc[lvl].p, st);
            return;
        }
        const int t0 = p.tile_off[lo], t1 = p.tile_off[hi + 1];
        if (t1 == t0) return;
        int kpmax = 0;
        for (int lvl = lo; lvl <= hi; ++lvl) kpmax = std::max(kpmax, o.lv[lvl].set->kp);
        const int ntl = t1 - t0;
        const int64_t nblk = p.m2l_xsplit ? 8 * ceil_div(ntl, 8 / p.nsplit) : int64_t(ntl) * p.nsplit;
        dim3 gr(unsigned(nblk), unsigned(ceil_div(kpmax, 64)), unsigned(ceil_div(r, p.rc_m2l)));
        if (o.precision != BBFMM_M2L_FP32) {
            M2LArgsLP g{};
            for (int lvl = lo; lvl <= hi; ++lvl) {
                const OpSet &set = *o.lv[lvl].set;
                g.lv[lvl] = M2LLevelLP{p.Mh16[lvl].p, p.Ml16[lvl].p, p.Msinv[lvl].p, p.Fh[lvl].p,
                                       o.precision == BBFMM_M2L_BF16X3 ? set.Chi.p : set.C16.p,
                                       set.Clo.p, set.Cinv.p, t.lv[lvl].itab.p,
                                       t.lv[lvl].oct_cells.p, set.kp, int64_t(t.lv[lvl].C) * r};
            }
            g.tiles = p.tiles.p;
            g.masks = p.masks.p;
            g.tables = t.tables.p;
            g.r = r;
            g.rc = p.rc_m2l;
            g.tpt = p.tpt;
            g.nsplit = p.nsplit;
            g.tile0 = t0;
            g.ntiles = ntl;
            g.xsplit = p.m2l_xsplit ? 1 : 0;
            if (o.precision == BBFMM_M2L_BF16X3)
                k_m2l_lp<BBFMM_M2L_BF16X3><<<gr, kThreads, p.m2l_pad_lds, st>>>(g);
            else
                k_m2l_lp<BBFMM_M2L_FP16_SCALED><<<gr, kThreads, p.m2l_pad_lds, st>>>(g);
        } else {
            M2LArgs g{};
            for (int lvl = lo; lvl <= hi; ++lvl) {
                const OpSet &set = *o.lv[lvl].set;
                g.lv[lvl] = M2LLevel{p.Mh[lvl].p, p.Fh[lvl].p, set.C32.p, t.lv[lvl].itab.p,
                                     t.lv[lvl].oct_cells.p, set.kp, int64_t(t.lv[lvl].C) * r};
            }
            g.tiles = p.tiles.p;
            g.masks = p.masks.p;
            g.tables = t.tables.p;
            g.r = r;
            g.rc = p.rc_m2l;
            g.tpt = p.tpt;
            g.nsplit = p.nsplit;
            g.tile0 = t0;
            g.ntiles = ntl;
            g.xsplit = p.m2l_xsplit ? 1 : 0;
            bool full = r % p.rc_m2l == 0;
            for (int lvl = lo; lvl <= hi; ++lvl) full = full && o.lv[lvl].set->kp % 64 == 0;
            if (p.m2l_layout == 2) {
                if (full) k_m2l<2, true><<<gr, kThreads, p.m2l_pad_lds, st>>>(g);
                else k_m2l<2, false><<<gr, kThreads, p.m2l_pad_lds, st>>>(g);
            } else {
                if (full) k_m2l<4, true><<<gr, kThreads, p.m2l_pad_lds, st>>>(g);
                else k_m2l<4, false><<<gr, kThreads, p.m2l_pad_lds, st>>>(g);
            }
        }
        BB_LAUNCH_CHECK();
    };
    // the fused leaf pass already compressed level L and formed level L-1
    if (L >= 2 && !p.leaf_fused) compress(L, s);
    if (!p.m2l_early) {
        mark(BBFMM_STAGE_M2M);
        for (int lvl = L - 1; lvl >= 2; --lvl) {
            if (!(p.leaf_fused && lvl == L - 1)) m2m(lvl, s);
            compress(lvl, s);
        }
        mark(BBFMM_STAGE_M2L);
        if (L >= 2) m2l(2, L, s);
    } else {
        // each level's M2L starts as soon as its compressed multipoles
        // exist: the leaf level's at once on `s`, while the upward chain
        // (M2M + compression of levels L-1..2) runs on the plan's `up`
        // stream and hands each finished level to `s` with an event
        mark(BBFMM_STAGE_M2M);
        BB_HIP(hipEventRecord(p.lev_ev[L], s));
        BB_HIP(hipStreamWaitEvent(p.up, p.lev_ev[L], 0));
        if (ev) BB_HIP(hipEventRecord(ev[kEvUpBeg], p.up));
        for (int lvl = L - 1; lvl >= 2; --lvl) {
            if (!(p.leaf_fused && lvl == L - 1)) m2m(lvl, p.up);
            compress(lvl, p.up);
            BB_HIP(hipEventRecord(p.lev_ev[lvl], p.up));
        }
        if (ev) BB_HIP(hipEventRecord(ev[kEvUpEnd], p.up));
        mark(BBFMM_STAGE_M2L);
        m2l(L, L, s);
        for (int lvl = L - 1; lvl >= 2; --lvl) {
            BB_HIP(hipStreamWaitEvent(s, p.lev_ev[lvl], 0));
            m2l(lvl, lvl, s);
        }
    }
    mark(BBFMM_STAGE_DOWN);
    for (int lvl = 2; lvl <= L; ++lvl) {
        const LevelData &lv = t.lv[lvl];
        const OpSet &set = *o.lv[lvl].set;
        if (lvl > 2) {
            const LevelData &pa = t.lv[lvl - 1];
            switch (n) {
#define BB_L2L(NN) case NN: k_l2l_pen<NN><<<dim3(unsigned(pa.C), unsigned(ceil_div(r, Pencil<NN>::G))), \
                64, 0, s>>>(pa.cb.p, pa.ce.p, lv.keys.p, p.F[lvl - 1].p, o.cheb, r, mp, p.F[lvl].p); break;
            BB_L2L(2) BB_L2L(3) BB_L2L(4) BB_L2L(5) BB_L2L(6) BB_L2L(7) BB_L2L(8)
#undef BB_L2L
            }
            BB_LAUNCH_CHECK();
        }
        const int64_t R = int64_t(lv.C) * r;
        if (o.precision == BBFMM_M2L_FFT) {
            fft_inverse(n, p.Fc[lvl].p, R, float(o.lv[lvl].scale), lvl > 2, mp, p.F[lvl].p, s);
        } else {
            dim3 g(unsigned(ceil_div(R, 64)), unsigned(ceil_div(mp, 64)));
            k_gemm_nt<kOutF32><<<g, kThreads, 0, s>>>(p.Fh[lvl].p, set.kp, p.nsplit, R * set.kp,
                                                     set.U32.p, set.kp, p.F[lvl].p, mp, R, mp,
                                                     set.kp, float(o.lv[lvl].scale),
                                                     lvl > 2 ? 1.f : 0.f, nullptr, nullptr,
                                                     nullptr, 0);
            BB_LAUNCH_CHECK();
        }
        if (t.adaptive && lv.nx_cells > 0) {
            // P2L: the X leaves' points into this level's local expansions
            Geo gl = geo;
            gl.h = float(t.half_width(lvl));
            gl.inv_h = 1.0f / gl.h;
            const float cs = coord_scale(t.params.kernel_id, t.params.kernel_param);
            const LevelData &fl = t.leaves();
            // columns per wave: one, or blocks of 16 (on MFMA with the MFMA near field)
            const int rc = r == 1 ? 1 : 16;
            dim3 g(unsigned(lv.nx_cells), unsigned(ceil_div(r, rc)));
#define BB_P2L_N(NN, KK)                                                                              \
            if (rc == 1) k_p2l<NN, KK, 1><<<g, 64, 0, s>>>(BB_P2L_ARGS);                              \
            else if (p.p2p_mfma) k_p2l_mfma<NN, KK><<<g, 64, 0, s>>>(BB_P2L_ARGS);                    \
            else k_p2l<NN, KK, 16><<<g, 64, 0, s>>>(BB_P2L_ARGS);
#define BB_P2L(KK)                                                                                    \
            switch (n) {                                                                              \
            case 2: BB_P2L_N(2, KK) break;                                                            \
            case 3: BB_P2L_N(3, KK) break;                                                            \
            case 4: BB_P2L_N(4, KK) break;                                                            \
            case 5: BB_P2L_N(5, KK) break;                                                            \
            case 6: BB_P2L_N(6, KK) break;                                                            \
            case 7: BB_P2L_N(7, KK) break;                                                            \
            default: BB_P2L_N(8, KK) break;                                                           \
            }
#define BB_P2L_ARGS lv.x_cells.p, lv.x_off.p, lv.x_leaf.p, fl.pb.p, fl.pe.p, lv.keys.p, t.xs.p, \
                    t.ys.p, t.zs.p, p.sig_s.p, p.ld_s, gl, o.cheb, cs, r, mp, p.F[lvl].p
            switch (t.params.kernel_id) {
            case BBFMM_K_INV_R: BB_P2L(BBFMM_K_INV_R) break;
            case BBFMM_K_EXP: BB_P2L(BBFMM_K_EXP) break;
            case BBFMM_K_GAUSS: BB_P2L(BBFMM_K_GAUSS) break;
            case BBFMM_K_DIPOLE_X: BB_P2L(BBFMM_K_DIPOLE_X) break;
            default: BB_P2L(BBFMM_K_POLY_TEST) break;
            }
#undef BB_P2L_ARGS
#undef BB_P2L
#undef BB_P2L_N
            BB_LAUNCH_CHECK();
        }
    }
    if (L >= 2 && !t.adaptive) FL = p.F[L].p;
    mark(BBFMM_STAGE_P2P);
    if (t.adaptive) {
        // near field over the U lists, then L2P and M2P added at every leaf
        if (p.overlap) {
            BB_HIP(hipStreamWaitEvent(s, p.join, 0));
            if (ev) BB_HIP(hipEventRecord(ev[kEvJoined], s));
        } else {
            near_field(nullptr, s);
        }
        if (L >= 2) leaf_far(p, geo, phi, s);
    } else if (p.overlap || p.p2p_pack) {
        if (p.overlap) {
            BB_HIP(hipStreamWaitEvent(s, p.join, 0));
            if (ev) BB_HIP(hipEventRecord(ev[kEvJoined], s));
        } else {
            near_field(nullptr, s);
        }
        if (FL != nullptr) {
            const LevelData &leaf = t.lv[L];
            switch (n) {
#define BB_L2P(NN) case NN: k_l2p<NN><<<grid(t.n), kThreads, 0, s>>>(t.xs.p, t.ys.p, t.zs.p, p.pleaf.p, \
                leaf.keys.p, t.perm.p, t.n, t.n_out(), r, FL, mp, geo, o.cheb, phi); break;
            BB_L2P(2) BB_L2P(3) BB_L2P(4) BB_L2P(5) BB_L2P(6) BB_L2P(7) BB_L2P(8)
#undef BB_L2P
            }
            BB_LAUNCH_CHECK();
        }
    } else {
        near_field(FL, s);
    }
    mark(BBFMM_NUM_STAGES);
}

}  // namespace

}  // namespace bbfmm

bbfmm_ops::~bbfmm_ops() { bbfmm::plan_cache_destroy(cache); }
