// M2L on equally spaced interpolation nodes by the FFT (Section 2.5, fast
// M2L translation).
//
// With the nodes s_m = -1 + 2m/(n-1) on every axis, the operator between a
// target cell and a source cell at transfer vector t,
//     K_t[i][j] = K(h s_i, h (2t + s_j)),
// depends on i and j only through the per-axis differences d = i - j, so
// K_t is a three-level Toeplitz matrix with (2n-1)^3 distinct entries
//     g_t(d) = K(h (delta d - 2t)),   delta = 2/(n-1),   d in (-n, n)^3.
// The product F = K_t M is the linear convolution F[i] = sum_j g_t(i-j) M[j];
// embedded in a circulant of size P = 2n >= 2n-1 per axis it is the cyclic
// convolution of the P^3 array G_t (g_t placed at d mod P, zero elsewhere)
// with M zero-padded to P^3, i.e. pointwise multiplication of their discrete
// Fourier transforms.  A real array's transform is determined by the half
// k3 in [0, P/2]; Q = (P/2 + 1) P^2 complex values per (cell, column).
//
//   forward   Mhat[cell][c][k3][k2][k1] = DFT of M (x fastest), one pass per
//             axis over the nonzero input lines only
//   M2L       Fhat[a] = sum over the interaction list of Ghat_t * Mhat[b]
//             (pointwise complex multiply-add over the Q frequencies)
//   inverse   F += scale * IDFT(Fhat) restricted to the n^3 nodes
//             (x and y inverse passes, then the Hermitian sum along z)
//
// Transforms are direct sums with twiddles from a table computed in double
// on the host (P <= 16), so each pass is a few multiply-adds per output.
// The operator spectra Ghat_t are computed once in FP64 on the GPU (the plain
// DFT definition) and stored as FP32 complex.
#include "common.h"

#include <vector>

namespace bbfmm {
namespace {

constexpr int kThreads = 256;
constexpr int kMaxP = 2 * kMaxOrder;

inline int grid(int64_t n) { return int(ceil_div(n, kThreads)); }

// cos / sin of 2 pi j / P, j < P
struct Twiddle {
    float c[kMaxP], s[kMaxP];
};

Twiddle make_twiddle(int P) {
    Twiddle w{};
    for (int j = 0; j < P; ++j) {
        const double a = 2.0 * M_PI * double(j) / double(P);
        w.c[j] = float(std::cos(a));
        w.s[j] = float(std::sin(a));
    }
    return w;
}

// Forward transform of one (cell, column) row of M per workgroup.
// exp(-2 pi i j k / P) = c[jk mod P] - i s[jk mod P].
template <int N>
__global__ void __launch_bounds__(kThreads)
k_fft_forward(const float *M, int mp, int64_t rows, Twiddle w, float2 *Mhat) {
    constexpr int P = 2 * N, H = P / 2 + 1, Q = H * P * P, m = N * N * N;
    __shared__ float x[m];
    __shared__ float2 A[N * N * P];      // [i3][i2][k1]
    __shared__ float2 B[N * P * P];      // [i3][k2][k1]
    const int64_t row = blockIdx.x;
    if (row >= rows) return;
    const int tid = threadIdx.x;
    for (int i = tid; i < m; i += kThreads) x[i] = M[row * mp + i];
    __syncthreads();
    for (int e = tid; e < N * N * P; e += kThreads) {
        const int k1 = e % P, l = e / P;                 // l = i3 * N + i2
        float re = 0.f, im = 0.f;
#pragma unroll
        for (int i1 = 0; i1 < N; ++i1) {
            const int q = (i1 * k1) % P;
            const float v = x[l * N + i1];
            re = __fmaf_rn(v, w.c[q], re);
            im = __fmaf_rn(-v, w.s[q], im);
        }
        A[e] = make_float2(re, im);
    }
    __syncthreads();
    for (int e = tid; e < N * P * P; e += kThreads) {
        const int k1 = e % P, k2 = (e / P) % P, i3 = e / (P * P);
        float re = 0.f, im = 0.f;
#pragma unroll
        for (int i2 = 0; i2 < N; ++i2) {
            const int q = (i2 * k2) % P;
            const float2 v = A[(i3 * N + i2) * P + k1];
            // (v.x + i v.y) (c - i s)
            re = __fmaf_rn(v.x, w.c[q], __fmaf_rn(v.y, w.s[q], re));
            im = __fmaf_rn(v.y, w.c[q], __fmaf_rn(-v.x, w.s[q], im));
        }
        B[e] = make_float2(re, im);
    }
    __syncthreads();
    float2 *out = Mhat + row * Q;
    for (int e = tid; e < Q; e += kThreads) {
        const int k12 = e % (P * P), k3 = e / (P * P);
        float re = 0.f, im = 0.f;
#pragma unroll
        for (int i3 = 0; i3 < N; ++i3) {
            const int q = (i3 * k3) % P;
            const float2 v = B[i3 * P * P + k12];
            re = __fmaf_rn(v.x, w.c[q], __fmaf_rn(v.y, w.s[q], re));
            im = __fmaf_rn(v.y, w.c[q], __fmaf_rn(-v.x, w.s[q], im));
        }
        out[e] = make_float2(re, im);
    }
}

// Inverse transform of one row of Fhat restricted to the n^3 nodes:
// F[row][node] = scale * IDFT + (accumulate ? F[row][node] : 0); padding
// nodes m..mp are written as zero when not accumulating.
// exp(+2 pi i j k / P) = c + i s.
template <int N>
__global__ void __launch_bounds__(kThreads)
k_fft_inverse(const float2 *Fhat, int64_t rows, Twiddle w, float scale, int accumulate, int mp,
              float *F) {
    constexpr int P = 2 * N, H = P / 2 + 1, Q = H * P * P, m = N * N * N;
    __shared__ float2 X[Q];              // [k3][k2][k1]
    __shared__ float2 B1[H * P * N];     // [k3][k2][l1]
    __shared__ float2 B2[H * N * N];     // [k3][l2][l1]
    const int64_t row = blockIdx.x;
    if (row >= rows) return;
    const int tid = threadIdx.x;
    for (int e = tid; e < Q; e += kThreads) X[e] = Fhat[row * Q + e];
    __syncthreads();
    for (int e = tid; e < H * P * N; e += kThreads) {
        const int l1 = e % N, r = e / N;                 // r = k3 * P + k2
        float re = 0.f, im = 0.f;
#pragma unroll
        for (int k1 = 0; k1 < P; ++k1) {
            const int q = (k1 * l1) % P;
            const float2 v = X[r * P + k1];
            // (v.x + i v.y) (c + i s)
            re = __fmaf_rn(v.x, w.c[q], __fmaf_rn(-v.y, w.s[q], re));
            im = __fmaf_rn(v.y, w.c[q], __fmaf_rn(v.x, w.s[q], im));
        }
        B1[e] = make_float2(re, im);
    }
    __syncthreads();
    for (int e = tid; e < H * N * N; e += kThreads) {
        const int l1 = e % N, l2 = (e / N) % N, k3 = e / (N * N);
        float re = 0.f, im = 0.f;
#pragma unroll
        for (int k2 = 0; k2 < P; ++k2) {
            const int q = (k2 * l2) % P;
            const float2 v = B1[(k3 * P + k2) * N + l1];
            re = __fmaf_rn(v.x, w.c[q], __fmaf_rn(-v.y, w.s[q], re));
            im = __fmaf_rn(v.y, w.c[q], __fmaf_rn(v.x, w.s[q], im));
        }
        B2[e] = make_float2(re, im);
    }
    __syncthreads();
    const float norm = scale / float(P * P * P);
    float *out = F + row * mp;
    for (int e = tid; e < mp; e += kThreads) {
        if (e >= m) {
            if (!accumulate) out[e] = 0.f;
            continue;
        }
        const int l12 = e % (N * N), l3 = e / (N * N);
        // Hermitian along k3: k3 = 0 and P/2 once, the others twice
        float acc = B2[l12].x;
#pragma unroll
        for (int k3 = 1; k3 < P / 2; ++k3) {
            const int q = (k3 * l3) % P;
            const float2 v = B2[k3 * N * N + l12];
            acc = __fmaf_rn(2.f, __fmaf_rn(v.x, w.c[q], -v.y * w.s[q]), acc);
        }
        const float2 v = B2[(P / 2) * N * N + l12];
        acc = __fmaf_rn(v.x, (l3 & 1) ? -1.f : 1.f, acc);
        const float val = acc * norm;
        out[e] = accumulate ? out[e] + val : val;
    }
}

// Fhat[a][c] = sum over the interaction list of a of Ghat_t * Mhat[b][c]
// (all Q frequencies); one workgroup per (target cell, column), threads
// over frequencies.
__global__ void __launch_bounds__(kThreads)
k_m2l_fft(const float2 *Mhat, const float2 *Ghat, const int32_t *itab, const uint64_t *keys,
          const int32_t *slot_t, int r, int Q, float2 *Fhat) {
    const int a = blockIdx.x, c = blockIdx.y;
    const int oct = int(keys[a] & 7u);
    const int32_t *it = itab + int64_t(a) * kSlots;
    const int32_t *st = slot_t + oct * kSlots;
    for (int q0 = 0; q0 < Q; q0 += kThreads) {
        const int q = q0 + threadIdx.x;
        const bool ok = q < Q;
        float re = 0.f, im = 0.f;
        for (int j = 0; j < kSlots; ++j) {
            const int b = it[j];
            if (b < 0) continue;                      // uniform over the workgroup
            if (!ok) continue;
            const float2 g = Ghat[int64_t(st[j]) * Q + q];
            const float2 v = Mhat[(int64_t(b) * r + c) * Q + q];
            re = __fmaf_rn(g.x, v.x, __fmaf_rn(-g.y, v.y, re));
            im = __fmaf_rn(g.x, v.y, __fmaf_rn(g.y, v.x, im));
        }
        if (ok) Fhat[(int64_t(a) * r + c) * Q + q] = make_float2(re, im);
    }
}

// Spatially blocked form of the same sums (level-uniform trees).  One
// workgroup per (block of 4 x 4 x 4 target cells, slice of kFq frequencies,
// column): the slice of the 8 x 8 x 8 source halo's spectra and of the 316
// operator spectra is staged in LDS once, so each staged source value serves
// every target of the block that has it in its list instead of being
// gathered again per target.  Thread (q, o, k): frequency q of the slice,
// octant o, part k of the 189 slots; it accumulates the block's eight
// targets of octant o (one per parent), which share the transfer vector of
// every slot, so one operator value serves eight products.  The parts'
// partial sums are added in part order.  A slot whose source cell does not
// exist reads a zero halo entry.
constexpr int kHalo = 512;          // 8 x 8 x 8 source cells

template <int kFq>
__global__ void __launch_bounds__(kThreads)
k_m2l_fft_blk(const float2 *Mhat, const float2 *Ghat, const int32_t *btgt, const int32_t *bhalo,
              const int32_t *slots, int r, int Q, float2 *Fhat) {
    constexpr int kRow = kFq + 1;               // LDS row of one halo cell's slice (padded)
    constexpr int kParts = kThreads / (8 * kFq); // slot ranges, summed in order
    static_assert(kParts * 64 * kFq <= kHalo * kRow + kNumT * kFq, "partial sums reuse the slices");
    __shared__ float2 stage[kHalo * kRow + kNumT * kFq];
    float2 *hs = stage, *gs = stage + kHalo * kRow;
    __shared__ int32_t sb[8 * kSlots];        // FftBlocks::slots
    const int blk = blockIdx.x, q0 = blockIdx.y * kFq, c = blockIdx.z;
    const int tid = threadIdx.x;
    const int32_t *halo = bhalo + int64_t(blk) * kHalo;
    // Every staging load is issued before the first LDS store (addresses
    // clamped in bounds, values selected afterwards), so the workgroup waits
    // for one round of loads rather than one per element.
    constexpr int kHn = kHalo * kFq / kThreads;
    constexpr int kGn = (kNumT * kFq + kThreads - 1) / kThreads;
    constexpr int kSn = (8 * kSlots + kThreads - 1) / kThreads;
    int32_t hb[kHn];
#pragma unroll
    for (int i = 0; i < kHn; ++i) hb[i] = halo[(tid + i * kThreads) / kFq];
    float2 hv[kHn], gv[kGn];
    int32_t tv[kSn];
#pragma unroll
    for (int i = 0; i < kHn; ++i) {
        const int qq = min(q0 + (tid + i * kThreads) % kFq, Q - 1);
        hv[i] = Mhat[(int64_t(max(hb[i], 0)) * r + c) * Q + qq];
    }
#pragma unroll
    for (int i = 0; i < kGn; ++i) {
        const int e = min(tid + i * kThreads, kNumT * kFq - 1);
        gv[i] = Ghat[int64_t(e / kFq) * Q + min(q0 + e % kFq, Q - 1)];
    }
#pragma unroll
    for (int i = 0; i < kSn; ++i) tv[i] = slots[min(tid + i * kThreads, 8 * kSlots - 1)];
#pragma unroll
    for (int i = 0; i < kHn; ++i) {
        const int e = tid + i * kThreads;
        const bool ok = hb[i] >= 0 && q0 + e % kFq < Q;
        hs[(e / kFq) * kRow + e % kFq] = ok ? hv[i] : make_float2(0.f, 0.f);
    }
#pragma unroll
    for (int i = 0; i < kGn; ++i) {
        const int e = tid + i * kThreads;
        if (e < kNumT * kFq) gs[e] = q0 + e % kFq < Q ? gv[i] : make_float2(0.f, 0.f);
    }
#pragma unroll
    for (int i = 0; i < kSn; ++i) {
        const int e = tid + i * kThreads;
        if (e < 8 * kSlots) sb[e] = tv[i];
    }
    __syncthreads();
    const int q = tid % kFq, o = (tid / kFq) % 8, k = tid / (8 * kFq);
    float2 acc[8];
#pragma unroll
    for (int p = 0; p < 8; ++p) acc[p] = make_float2(0.f, 0.f);
    const int j0 = k * kSlots / kParts, j1 = (k + 1) * kSlots / kParts;
    for (int j = j0; j < j1; ++j) {
        const int v = sb[o * kSlots + j];
        const float2 g = gs[(v & 0xffff) * kFq + q];
        const float2 *hrow = hs + (v >> 16) * kRow + q;
#pragma unroll
        for (int p = 0; p < 8; ++p) {
            const float2 m = hrow[(2 * (p & 1) + 16 * ((p >> 1) & 1) + 128 * (p >> 2)) * kRow];
            acc[p].x = __fmaf_rn(g.x, m.x, __fmaf_rn(-g.y, m.y, acc[p].x));
            acc[p].y = __fmaf_rn(g.x, m.y, __fmaf_rn(g.y, m.x, acc[p].y));
        }
    }
    __syncthreads();                          // the staged slices are no longer read
    float2 *part = stage;                     // [k][target p * 8 + o][q]
#pragma unroll
    for (int p = 0; p < 8; ++p) part[(k * 64 + p * 8 + o) * kFq + q] = acc[p];
    __syncthreads();
    const int32_t *tg = btgt + int64_t(blk) * 64;
    for (int e = tid; e < 64 * kFq; e += kThreads) {
        const int l = e / kFq, qq = e % kFq;
        const int a = tg[l];
        if (a < 0 || q0 + qq >= Q) continue;
        float2 sum = part[e];
        for (int kk = 1; kk < kParts; ++kk) {
            const float2 v = part[kk * 64 * kFq + e];
            sum.x += v.x;
            sum.y += v.y;
        }
        Fhat[(int64_t(a) * r + c) * Q + q0 + qq] = sum;
    }
}

// ---------------------------------------------- operator spectra (FP64) ----
__device__ inline double kernel_f64(int kid, double a, double dx, double dy, double dz) {
    const double r2 = dx * dx + dy * dy + dz * dz;
    switch (kid) {
    case BBFMM_K_INV_R: return r2 > 0.0 ? 1.0 / sqrt(r2) : 0.0;
    case BBFMM_K_EXP: return exp(-sqrt(r2) / a);
    case BBFMM_K_GAUSS: return exp(-r2 / (a * a));
    case BBFMM_K_DIPOLE_X: return r2 > 0.0 ? dx / (r2 * sqrt(r2)) : 0.0;
    case BBFMM_K_POLY_TEST: {
        const double u[3] = {dx / a, dy / a, dz / a};
        double p = 1.0;
        for (int d = 0; d < 3; ++d)
            p *= 1.0 + u[d] / 2.0 - u[d] * u[d] / 3.0 + u[d] * u[d] * u[d] / 5.0;
        return p;
    }
    default: return 0.0;
    }
}

// G[t][e3][e2][e1] = g_t(d), d_x = e1 (e1 < n) or e1 - P (e1 > P - n), 0 in
// the gap; g_t(d) = K(h (delta d - 2t)) (target minus source).
__global__ void __launch_bounds__(kThreads)
k_fft_sample(int kid, double a, int n, int P, double h, const int32_t *tvec, double *G) {
    const int64_t P3 = int64_t(P) * P * P;
    const int64_t g = int64_t(blockIdx.x) * kThreads + threadIdx.x;
    if (g >= kNumT * P3) return;
    const int t = int(g / P3);
    const int e = int(g % P3);
    const int e1 = e % P, e2 = (e / P) % P, e3 = e / (P * P);
    const int ev[3] = {e1, e2, e3};
    const double delta = 2.0 / double(n - 1);
    double diff[3];
    for (int d = 0; d < 3; ++d) {
        int dd;
        if (ev[d] < n) dd = ev[d];
        else if (ev[d] > P - n) dd = ev[d] - P;
        else { G[g] = 0.0; return; }
        diff[d] = h * (delta * double(dd) - 2.0 * double(tvec[3 * t + d]));
    }
    G[g] = kernel_f64(kid, a, diff[0], diff[1], diff[2]);
}

// Ghat[t][k3][k2][k1] = sum_e G[t][e] exp(-2 pi i (k . e) / P), k3 <= P/2,
// as FP32 complex (the plain definition, one output per thread, FP64)
__global__ void __launch_bounds__(kThreads)
k_fft_spectrum(const double *G, int P, float2 *Ghat) {
    const int H = P / 2 + 1;
    const int64_t Q = int64_t(H) * P * P, P3 = int64_t(P) * P * P;
    const int64_t g = int64_t(blockIdx.x) * kThreads + threadIdx.x;
    if (g >= kNumT * Q) return;
    const int t = int(g / Q);
    const int q = int(g % Q);
    const int k1 = q % P, k2 = (q / P) % P, k3 = q / (P * P);
    const double *src = G + t * P3;
    double re = 0.0, im = 0.0;
    for (int e3 = 0; e3 < P; ++e3)
        for (int e2 = 0; e2 < P; ++e2)
            for (int e1 = 0; e1 < P; ++e1) {
                const int ph = (k1 * e1 + k2 * e2 + k3 * e3) % P;
                double s, c;
                sincospi(2.0 * double(ph) / double(P), &s, &c);
                const double v = src[(e3 * P + e2) * P + e1];
                re += v * c;
                im -= v * s;
            }
    Ghat[g] = make_float2(float(re), float(im));
}

}  // namespace

int fft_size(int n) { return 2 * n; }
int fft_freqs(int n) { return (n + 1) * (2 * n) * (2 * n); }   // (P/2 + 1) P^2

void fft_operator_spectra(int kid, double a, int n, double h, const int32_t *tvec, DBuf<float2> &Ghat,
                          hipStream_t s) {
    const int P = fft_size(n);
    const int64_t P3 = int64_t(P) * P * P, Q = fft_freqs(n);
    DBuf<double> G(size_t(kNumT * P3));
    k_fft_sample<<<grid(kNumT * P3), kThreads, 0, s>>>(kid, a, n, P, h, tvec, G.p);
    BB_LAUNCH_CHECK();
    Ghat.alloc(size_t(kNumT * Q));
    k_fft_spectrum<<<grid(kNumT * Q), kThreads, 0, s>>>(G.p, P, Ghat.p);
    BB_LAUNCH_CHECK();
    BB_HIP(hipStreamSynchronize(s));
}

void fft_forward(int n, const float *M, int mp, int64_t rows, float2 *Mhat, hipStream_t s) {
    if (rows == 0) return;
    const Twiddle w = make_twiddle(fft_size(n));
    switch (n) {
#define BB_FWD(NN) case NN: k_fft_forward<NN><<<unsigned(rows), kThreads, 0, s>>>(M, mp, rows, w, Mhat); break;
    BB_FWD(2) BB_FWD(3) BB_FWD(4) BB_FWD(5) BB_FWD(6) BB_FWD(7) BB_FWD(8)
#undef BB_FWD
    default: fail(BBFMM_ERR_INTERNAL, "no FFT for order %d", n);
    }
    BB_LAUNCH_CHECK();
}

void fft_inverse(int n, const float2 *Fhat, int64_t rows, float scale, bool accumulate, int mp,
                 float *F, hipStream_t s) {
    if (rows == 0) return;
    const Twiddle w = make_twiddle(fft_size(n));
    switch (n) {
#define BB_INV(NN) case NN: k_fft_inverse<NN><<<unsigned(rows), kThreads, 0, s>>>(Fhat, rows, w, \
        scale, accumulate ? 1 : 0, mp, F); break;
    BB_INV(2) BB_INV(3) BB_INV(4) BB_INV(5) BB_INV(6) BB_INV(7) BB_INV(8)
#undef BB_INV
    default: fail(BBFMM_ERR_INTERNAL, "no FFT for order %d", n);
    }
    BB_LAUNCH_CHECK();
}

void fft_m2l(int n, const float2 *Mhat, const float2 *Ghat, const int32_t *itab,
             const uint64_t *keys, const int32_t *slot_t, int64_t cells, int r, float2 *Fhat,
             hipStream_t s) {
    if (cells == 0) return;
    k_m2l_fft<<<dim3(unsigned(cells), unsigned(r)), kThreads, 0, s>>>(Mhat, Ghat, itab, keys, slot_t, r,
                                                                      fft_freqs(n), Fhat);
    BB_LAUNCH_CHECK();
}


// Host side: the level's keys are ascending Morton keys, so a block's cells
// are one run of equal key >> 6.  Halo cells are found in a dense grid of
// the level (levels up to 8) or by binary search in the keys.
void fft_build_blocks(const uint64_t *keys, int32_t C, int lvl, FftBlocks &b, hipStream_t s) {
    std::vector<uint64_t> k(size_t(std::max(C, 0)));
    if (C > 0) {
        BB_HIP(hipMemcpyAsync(k.data(), keys, size_t(C) * sizeof(uint64_t), hipMemcpyDeviceToHost, s));
        BB_HIP(hipStreamSynchronize(s));
    }
    auto coord = [](uint64_t key, int d) {
        uint32_t v = 0;
        for (int i = 0; i < 21; ++i) v |= uint32_t((key >> (3 * i + d)) & 1u) << i;
        return int(v);
    };
    auto key_of = [](int x, int y, int z) {
        uint64_t key = 0;
        for (int i = 0; i < 21; ++i)
            key |= (uint64_t((x >> i) & 1) << (3 * i)) | (uint64_t((y >> i) & 1) << (3 * i + 1)) |
                   (uint64_t((z >> i) & 1) << (3 * i + 2));
        return key;
    };
    const int64_t lim = int64_t(1) << lvl;
    const bool dense = lvl <= 8;
    std::vector<int32_t> grid;
    if (dense) {
        grid.assign(size_t(lim * lim * lim), -1);
        for (int32_t a = 0; a < C; ++a)
            grid[size_t((coord(k[a], 2) * lim + coord(k[a], 1)) * lim + coord(k[a], 0))] = a;
    }
    auto find = [&](int x, int y, int z) -> int32_t {
        if (x < 0 || y < 0 || z < 0 || x >= lim || y >= lim || z >= lim) return -1;
        if (dense) return grid[size_t((z * lim + y) * lim + x)];
        const uint64_t key = key_of(x, y, z);
        const auto it = std::lower_bound(k.begin(), k.end(), key);
        return (it != k.end() && *it == key) ? int32_t(it - k.begin()) : -1;
    };
    std::vector<int32_t> tgt, halo;
    for (int32_t a = 0; a < C;) {
        const uint64_t bk = k[a] >> 6;
        tgt.insert(tgt.end(), 64, -1);
        int32_t *tb = tgt.data() + tgt.size() - 64;
        for (; a < C && (k[a] >> 6) == bk; ++a) tb[k[a] & 63] = a;
        const int bx = 4 * coord(bk, 0), by = 4 * coord(bk, 1), bz = 4 * coord(bk, 2);
        for (int hz = 0; hz < 8; ++hz)
            for (int hy = 0; hy < 8; ++hy)
                for (int hx = 0; hx < 8; ++hx) halo.push_back(find(bx - 2 + hx, by - 2 + hy, bz - 2 + hz));
    }
    // the source of slot j of the target at (2 px + ox, 2 py + oy, 2 pz + oz)
    // in the block is that cell plus t: halo cell base(o, t) + 2 px + 16 py
    // + 128 pz with base(o, t) = ((oz + tz + 2) * 8 + (oy + ty + 2)) * 8 +
    // ox + tx + 2, each term in [0, 5] for the slots of octant o
    const TransferTables &tt = transfer_tables();
    std::vector<int32_t> slots(8 * kSlots);
    for (int o = 0; o < 8; ++o)
        for (int j = 0; j < kSlots; ++j) {
            const int t = tt.slot_t[o][j];
            const int hx = (o & 1) + tt.tvec[t][0] + 2, hy = ((o >> 1) & 1) + tt.tvec[t][1] + 2,
                      hz = (o >> 2) + tt.tvec[t][2] + 2;
            slots[size_t(o) * kSlots + j] = t | (((hz * 8 + hy) * 8 + hx) << 16);
        }
    b.nblk = int32_t(tgt.size() / 64);
    b.tgt.alloc(tgt.size());
    b.halo.alloc(halo.size());
    b.slots.alloc(slots.size());
    BB_HIP(hipMemcpyAsync(b.slots.p, slots.data(), slots.size() * sizeof(int32_t), hipMemcpyHostToDevice, s));
    if (b.nblk > 0) {
        BB_HIP(hipMemcpyAsync(b.tgt.p, tgt.data(), tgt.size() * sizeof(int32_t), hipMemcpyHostToDevice, s));
        BB_HIP(hipMemcpyAsync(b.halo.p, halo.data(), halo.size() * sizeof(int32_t), hipMemcpyHostToDevice, s));
    }
    BB_HIP(hipStreamSynchronize(s));
}

void fft_m2l_blocks(int n, const float2 *Mhat, const float2 *Ghat, const FftBlocks &b, int r,
                    float2 *Fhat, hipStream_t s) {
    if (b.nblk == 0) return;
    const int Q = fft_freqs(n);
    BB_REQUIRE(r >= 1 && r <= 65535, "FFT M2L: r out of range");
    constexpr int F = 4;        // frequencies per workgroup (measured: 4 beats 2 and 8)
    k_m2l_fft_blk<F><<<dim3(unsigned(b.nblk), unsigned(ceil_div(Q, F)), unsigned(r)), kThreads, 0, s>>>(
        Mhat, Ghat, b.tgt.p, b.halo.p, b.slots.p, r, Q, Fhat);
    BB_LAUNCH_CHECK();
}

}  // namespace bbfmm
