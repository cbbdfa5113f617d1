// M2L operator precompute on the GPU, in FP64 (Sections 2.3 and 2.5).
//
//   K_t[i][j] = K(h s_i, h (2t + s_j))     316 operators of n^3 x n^3
//   G_fat  = sum_t K_t K_t^T,  G_thin = sum_t K_t^T K_t
//   G = Q diag(lambda) Q^T by a parallel cyclic Jacobi eigensolver
//   singular values of the fat / thin concatenations = sqrt(lambda)
//   k = max(#{sigma > eps sigma_1} of both), U / V = leading eigenvectors
//   C_t = U^T K_t V, then cast to float (zero-padded to the MFMA tile)
//
// The left singular vectors of [K_t1 K_t2 ...] are the eigenvectors of
// G_fat and the right singular vectors of [K_t1; K_t2; ...] those of G_thin,
// so the compression never forms the 316 n^3-wide matrices.  Forming G
// squares the condition number; singular values at the eps = 1e-5 cut sit
// near 1e-10 of the largest eigenvalue, far above FP64 round-off, so the
// rank and the retained subspace are resolved.
#include <cmath>

#include "common.h"

namespace bbfmm {
namespace {

constexpr int kThreads = 256;
constexpr double kMinSvdEps = 1e-7;    // smallest relative SVD threshold the Gram route resolves

__device__ inline double kernel_eval_f64(int kid, double a, double dx, double dy, double dz) {
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

// Interpolation nodes (Chebyshev cos((2m+1) pi / 2n), or equally spaced
// -1 + 2m/(n-1) when `uniform`), barycentric weights and the two 1D child
// maps T[o][i][j] = l_i((2o-1)/2 + s_j/2) (the parent basis at child nodes).
__global__ void k_cheb(int n, int uniform, double *out) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double s[kMaxOrder];
    for (int m = 0; m < n; ++m)
        s[m] = uniform ? -1.0 + 2.0 * m / (n - 1) : cos((2.0 * m + 1.0) * M_PI / (2.0 * n));
    for (int m = 0; m < n; ++m) {
        double w = 1.0;
        for (int k = 0; k < n; ++k)
            if (k != m) w *= s[m] - s[k];
        out[m] = s[m];
        out[kMaxOrder + m] = 1.0 / w;
    }
    for (int o = 0; o < 2; ++o)
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j) {
                const double x = (2.0 * o - 1.0) / 2.0 + s[j] / 2.0;
                double l = 1.0;
                for (int k = 0; k < n; ++k)
                    if (k != i) l *= (x - s[k]) / (s[i] - s[k]);
                out[2 * kMaxOrder + (o * kMaxOrder + i) * kMaxOrder + j] = l;
            }
}

__global__ void __launch_bounds__(kThreads)
k_sample(int kid, double a, int n, double h, const double *cheb, const int32_t *tvec,
         double *K) {
    const int m = n * n * n;
    const int64_t g = int64_t(blockIdx.x) * kThreads + threadIdx.x;
    if (g >= int64_t(kNumT) * m * m) return;
    const int t = int(g / (int64_t(m) * m));
    const int i = int((g / m) % m), j = int(g % m);
    const double *s = cheb;
    const double xi[3] = {h * s[i % n], h * s[(i / n) % n], h * s[i / (n * n)]};
    const double yj[3] = {h * (2.0 * tvec[3 * t] + s[j % n]),
                          h * (2.0 * tvec[3 * t + 1] + s[(j / n) % n]),
                          h * (2.0 * tvec[3 * t + 2] + s[j / (n * n)])};
    K[g] = kernel_eval_f64(kid, a, xi[0] - yj[0], xi[1] - yj[1], xi[2] - yj[2]);
}

// C[b] (+)= sum over the K index of A_b(i,k) B_b(k,j); with `sum_batches`
// every batch accumulates into C[0].  Strides address any transpose.
struct GemmArgs {
    int M, N, K, batches, sum_batches;
    const double *A; int64_t sAb, sAi, sAk;
    const double *B; int64_t sBb, sBk, sBj;
    double *C; int64_t sCb, sCi, sCj;
};

__global__ void __launch_bounds__(kThreads) k_dgemm(GemmArgs g) {
    __shared__ double As[16][17], Bs[16][17];
    const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
    const int i = blockIdx.y * 16 + ty, j = blockIdx.x * 16 + tx;
    const int b0 = g.sum_batches ? 0 : blockIdx.z;
    const int b1 = g.sum_batches ? g.batches : blockIdx.z + 1;
    double acc = 0.0;
    for (int b = b0; b < b1; ++b) {
        const double *A = g.A + b * g.sAb;
        const double *B = g.B + b * g.sBb;
        for (int k0 = 0; k0 < g.K; k0 += 16) {
            const int ia = blockIdx.y * 16 + ty, ka = k0 + tx;
            As[ty][tx] = (ia < g.M && ka < g.K) ? A[ia * g.sAi + ka * g.sAk] : 0.0;
            const int kb = k0 + ty, jb = blockIdx.x * 16 + tx;
            Bs[ty][tx] = (kb < g.K && jb < g.N) ? B[kb * g.sBk + jb * g.sBj] : 0.0;
            __syncthreads();
#pragma unroll
            for (int kk = 0; kk < 16; ++kk) acc += As[ty][kk] * Bs[kk][tx];
            __syncthreads();
        }
    }
    if (i < g.M && j < g.N) g.C[b0 * g.sCb + i * g.sCi + j * g.sCj] = acc;
}

void dgemm(const GemmArgs &g, hipStream_t s) {
    dim3 grid(unsigned(ceil_div(g.N, 16)), unsigned(ceil_div(g.M, 16)),
              unsigned(g.sum_batches ? 1 : g.batches));
    k_dgemm<<<grid, kThreads, 0, s>>>(g);
    BB_LAUNCH_CHECK();
}

__global__ void __launch_bounds__(kThreads) k_identity(double *Q, int m) {
    const int64_t g = int64_t(blockIdx.x) * kThreads + threadIdx.x;
    if (g < int64_t(m) * m) Q[g] = (g / m == g % m) ? 1.0 : 0.0;
}

// Cyclic Jacobi on a symmetric m x m matrix A (row-major, overwritten; its
// diagonal ends as the eigenvalues), accumulating Q (columns = vectors).
// One workgroup; each round applies m/2 disjoint rotations chosen by the
// round-robin (circle) schedule, so every pair (p, q) is visited once per
// sweep.  Rotation: Golub & Van Loan's symmetric 2x2 Schur decomposition.
constexpr int kJacobiThreads = 1024;

__global__ void __launch_bounds__(kJacobiThreads)
k_jacobi(double *A, double *Q, int m, int max_sweeps, double rel_tol, int *sweeps_out) {
    __shared__ int sp[256], sq[256];
    __shared__ double sc[256], ss[256];
    __shared__ double red[2][kJacobiThreads];
    __shared__ int done;
    __shared__ double prev_off;
    const int tid = threadIdx.x;
    const int mp = m + (m & 1);          // even number of players
    const int np = mp / 2;
    int sweep = 0;
    if (tid == 0) { done = 0; prev_off = INFINITY; }
    __syncthreads();
    for (sweep = 0; sweep < max_sweeps; ++sweep) {
        // convergence: off-diagonal mass against the whole matrix
        double off = 0.0, all = 0.0;
        for (int64_t g = tid; g < int64_t(m) * m; g += kJacobiThreads) {
            const double v = A[g] * A[g];
            all += v;
            if (g / m != g % m) off += v;
        }
        red[0][tid] = off;
        red[1][tid] = all;
        __syncthreads();
        for (int st = kJacobiThreads / 2; st > 0; st >>= 1) {
            if (tid < st) { red[0][tid] += red[0][tid + st]; red[1][tid] += red[1][tid + st]; }
            __syncthreads();
        }
        if (tid == 0) {
            const double o = red[0][0], t = red[1][0];
            // converged, or stalled at round-off level
            done = (o <= rel_tol * rel_tol * t ||
                    (o <= 1e-22 * t && o >= 0.25 * prev_off)) ? 1 : 0;
            prev_off = o;
        }
        __syncthreads();
        if (done) break;
        for (int r = 0; r < mp - 1; ++r) {
            if (tid < np) {
                const int i = tid;
                int a = (i == 0) ? 0 : 1 + (i - 1 + r) % (mp - 1);
                int b = 1 + (mp - 2 - i + r) % (mp - 1);
                int p = a < b ? a : b, q = a < b ? b : a;
                double c = 1.0, s = 0.0;
                if (q < m) {
                    const double apq = A[int64_t(p) * m + q];
                    if (apq != 0.0) {
                        const double app = A[int64_t(p) * m + p], aqq = A[int64_t(q) * m + q];
                        const double tau = (aqq - app) / (2.0 * apq);
                        const double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
                        c = 1.0 / sqrt(1.0 + t * t);
                        s = t * c;
                    }
                }
                sp[i] = p; sq[i] = q < m ? q : -1; sc[i] = c; ss[i] = s;
            }
            __syncthreads();
            // rows: A <- J^T A
            for (int64_t g = tid; g < int64_t(np) * m; g += kJacobiThreads) {
                const int i = int(g / m), k = int(g % m);
                const int q = sq[i];
                if (q < 0) continue;
                const int p = sp[i];
                const double c = sc[i], s = ss[i];
                const double x = A[int64_t(p) * m + k], y = A[int64_t(q) * m + k];
                A[int64_t(p) * m + k] = c * x - s * y;
                A[int64_t(q) * m + k] = s * x + c * y;
            }
            __syncthreads();
            // columns: A <- A J, Q <- Q J
            for (int64_t g = tid; g < int64_t(np) * m; g += kJacobiThreads) {
                const int i = int(g / m), k = int(g % m);
                const int q = sq[i];
                if (q < 0) continue;
                const int p = sp[i];
                const double c = sc[i], s = ss[i];
                double x = A[int64_t(k) * m + p], y = A[int64_t(k) * m + q];
                A[int64_t(k) * m + p] = c * x - s * y;
                A[int64_t(k) * m + q] = s * x + c * y;
                x = Q[int64_t(k) * m + p];
                y = Q[int64_t(k) * m + q];
                Q[int64_t(k) * m + p] = c * x - s * y;
                Q[int64_t(k) * m + q] = s * x + c * y;
            }
            __syncthreads();
            // the rotated pair is zero by construction
            if (tid < np && sq[tid] >= 0 && ss[tid] != 0.0) {
                A[int64_t(sp[tid]) * m + sq[tid]] = 0.0;
                A[int64_t(sq[tid]) * m + sp[tid]] = 0.0;
            }
            __syncthreads();
        }
    }
    if (tid == 0) *sweeps_out = sweep;
}

// The same cyclic Jacobi spread over the chip for larger m: one sweep is
// m-1 rounds, each three launches -- the rotation angles of the round's m/2
// disjoint pairs (from the matrix as it stands), then the row updates
// A <- J^T A, then the column updates A <- A J and Q <- Q J, in which the
// rotated pair's off-diagonal entries are set to zero.  Every element of a
// launch has one writer (pairs are disjoint), so the result is the
// single-workgroup schedule's.
__global__ void __launch_bounds__(kThreads)
k_jac_angles(const double *A, int m, int mp, int round, int32_t *pq, double *cs) {
    const int np = mp / 2;
    const int i = blockIdx.x * kThreads + threadIdx.x;
    if (i >= np) return;
    const int a = (i == 0) ? 0 : 1 + (i - 1 + round) % (mp - 1);
    const int b = 1 + (mp - 2 - i + round) % (mp - 1);
    const int p = a < b ? a : b, q = a < b ? b : a;
    double c = 1.0, s = 0.0;
    if (q < m) {
        const double apq = A[int64_t(p) * m + q];
        if (apq != 0.0) {
            const double app = A[int64_t(p) * m + p], aqq = A[int64_t(q) * m + q];
            const double tau = (aqq - app) / (2.0 * apq);
            const double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
            c = 1.0 / sqrt(1.0 + t * t);
            s = t * c;
        }
    }
    pq[2 * i] = p;
    pq[2 * i + 1] = q < m ? q : -1;
    cs[2 * i] = c;
    cs[2 * i + 1] = s;
}

__global__ void __launch_bounds__(kThreads)
k_jac_rows(double *A, int m, int np, const int32_t *pq, const double *cs) {
    const int64_t g = int64_t(blockIdx.x) * kThreads + threadIdx.x;
    if (g >= int64_t(np) * m) return;
    const int i = int(g / m), k = int(g % m);
    const int q = pq[2 * i + 1];
    if (q < 0) return;
    const int p = pq[2 * i];
    const double c = cs[2 * i], s = cs[2 * i + 1];
    const double x = A[int64_t(p) * m + k], y = A[int64_t(q) * m + k];
    A[int64_t(p) * m + k] = c * x - s * y;
    A[int64_t(q) * m + k] = s * x + c * y;
}

__global__ void __launch_bounds__(kThreads)
k_jac_cols(double *A, double *Q, int m, int np, const int32_t *pq, const double *cs) {
    const int64_t g = int64_t(blockIdx.x) * kThreads + threadIdx.x;
    if (g >= int64_t(np) * m) return;
    const int i = int(g / m), k = int(g % m);
    const int q = pq[2 * i + 1];
    if (q < 0) return;
    const int p = pq[2 * i];
    const double c = cs[2 * i], s = cs[2 * i + 1];
    double x = A[int64_t(k) * m + p], y = A[int64_t(k) * m + q];
    double np_ = c * x - s * y, nq = s * x + c * y;
    if (s != 0.0) {                      // the rotated pair is zero by construction
        if (k == q) np_ = 0.0;           // A[q][p]
        if (k == p) nq = 0.0;            // A[p][q]
    }
    A[int64_t(k) * m + p] = np_;
    A[int64_t(k) * m + q] = nq;
    x = Q[int64_t(k) * m + p];
    y = Q[int64_t(k) * m + q];
    Q[int64_t(k) * m + p] = c * x - s * y;
    Q[int64_t(k) * m + q] = s * x + c * y;
}

// off-diagonal and total squared mass of A (one workgroup)
__global__ void __launch_bounds__(kJacobiThreads) k_offdiag(const double *A, int m, double *out) {
    __shared__ double red[2][kJacobiThreads];
    const int tid = threadIdx.x;
    double off = 0.0, all = 0.0;
    for (int64_t g = tid; g < int64_t(m) * m; g += kJacobiThreads) {
        const double v = A[g] * A[g];
        all += v;
        if (g / m != g % m) off += v;
    }
    red[0][tid] = off;
    red[1][tid] = all;
    __syncthreads();
    for (int st = kJacobiThreads / 2; st > 0; st >>= 1) {
        if (tid < st) { red[0][tid] += red[0][tid + st]; red[1][tid] += red[1][tid + st]; }
        __syncthreads();
    }
    if (tid == 0) { out[0] = red[0][0]; out[1] = red[1][0]; }
}

// m from which the multi-workgroup schedule is used
constexpr int kJacobiWideFrom = 96;

inline int jgrid(int64_t n) { return int((n + kThreads - 1) / kThreads); }

int jacobi_wide(double *A, double *Q, int m, int max_sweeps, double rel_tol, hipStream_t s) {
    const int mp = m + (m & 1), np = mp / 2;
    DBuf<int32_t> pq(size_t(2 * np));
    DBuf<double> cs(size_t(2 * np)), red(2);
    double prev_off = INFINITY;
    int sweep = 0;
    for (; sweep < max_sweeps; ++sweep) {
        k_offdiag<<<1, kJacobiThreads, 0, s>>>(A, m, red.p);
        BB_LAUNCH_CHECK();
        double h[2] = {0.0, 0.0};
        BB_HIP(hipMemcpyAsync(h, red.p, sizeof(h), hipMemcpyDeviceToHost, s));
        BB_HIP(hipStreamSynchronize(s));
        // converged, or stalled at round-off level (the single-workgroup rule)
        if (h[0] <= rel_tol * rel_tol * h[1] || (h[0] <= 1e-22 * h[1] && h[0] >= 0.25 * prev_off))
            break;
        prev_off = h[0];
        for (int rd = 0; rd < mp - 1; ++rd) {
            k_jac_angles<<<jgrid(np), kThreads, 0, s>>>(A, m, mp, rd, pq.p, cs.p);
            k_jac_rows<<<jgrid(int64_t(np) * m), kThreads, 0, s>>>(A, m, np, pq.p, cs.p);
            k_jac_cols<<<jgrid(int64_t(np) * m), kThreads, 0, s>>>(A, Q, m, np, pq.p, cs.p);
        }
        BB_LAUNCH_CHECK();
    }
    return sweep;
}

// eigenvalues (diagonal of A) in descending order -> sv = sqrt(max(l, 0)),
// order[c] = index of the c-th largest; count[0] = #{l > eps^2 l_max}
__global__ void __launch_bounds__(kThreads)
k_eig_order(const double *A, int m, double eps, int32_t *order, double *sv, int32_t *count) {
    double lmax = 0.0;
    for (int j = 0; j < m; ++j) lmax = fmax(lmax, A[int64_t(j) * m + j]);
    for (int i = threadIdx.x; i < m; i += kThreads) {
        const double li = A[int64_t(i) * m + i];
        int rank = 0;
        for (int j = 0; j < m; ++j) {
            const double lj = A[int64_t(j) * m + j];
            if (lj > li || (lj == li && j < i)) ++rank;
        }
        order[rank] = i;
        sv[rank] = sqrt(fmax(li, 0.0));
        if (lmax > 0.0 && li > eps * eps * lmax) atomicAdd(count, 1);
    }
}

__global__ void __launch_bounds__(kThreads)
k_select_columns(const double *Q, int m, const int32_t *order, int k, double *U) {
    const int64_t g = int64_t(blockIdx.x) * kThreads + threadIdx.x;
    if (g >= int64_t(m) * k) return;
    const int i = int(g / k), c = int(g % k);
    const int oc = order[c];
    U[g] = (oc >= 0 && oc < m) ? Q[int64_t(i) * m + oc] : 0.0;
}

__global__ void __launch_bounds__(kThreads)
k_cast_pad(const double *src, int rows, int cols, int pad_rows, int pad_cols, int batches,
           float *dst) {
    const int64_t g = int64_t(blockIdx.x) * kThreads + threadIdx.x;
    const int64_t per = int64_t(pad_rows) * pad_cols;
    if (g >= per * batches) return;
    const int64_t b = g / per;
    const int i = int((g % per) / pad_cols), j = int(g % pad_cols);
    dst[g] = (i < rows && j < cols) ? float(src[b * rows * cols + int64_t(i) * cols + j]) : 0.f;
}

// dst[kk][i] = src[i][kk] (src m x k) as a kp x mp array, zero outside
__global__ void __launch_bounds__(kThreads)
k_cast_pad_t(const double *src, int m, int k, int mp, int kp, float *dst) {
    const int64_t g = int64_t(blockIdx.x) * kThreads + threadIdx.x;
    if (g >= int64_t(kp) * mp) return;
    const int kk = int(g / mp), i = int(g % mp);
    dst[g] = (kk < k && i < m) ? float(src[int64_t(i) * k + kk]) : 0.f;
}

// bf16 round-to-nearest-even of a float, as raw bits
__device__ inline uint16_t bf16_bits(float x) {
    const __bf16 h = static_cast<__bf16>(x);
    return __builtin_bit_cast(uint16_t, h);
}
__device__ inline float bf16_value(uint16_t b) {
    return static_cast<float>(__builtin_bit_cast(__bf16, b));
}

// hi = bf16(c), lo = bf16(c - hi) of every operator entry (zero-padded)
__global__ void __launch_bounds__(kThreads)
k_split_bf16(const double *C, int k, int kp, int batches, uint16_t *hi, uint16_t *lo) {
    const int64_t g = int64_t(blockIdx.x) * kThreads + threadIdx.x;
    const int64_t per = int64_t(kp) * kp;
    if (g >= per * batches) return;
    const int64_t b = g / per;
    const int i = int((g % per) / kp), j = int(g % kp);
    const double c = (i < k && j < k) ? C[b * k * k + int64_t(i) * k + j] : 0.0;
    const uint16_t h = bf16_bits(float(c));
    hi[g] = h;
    lo[g] = bf16_bits(float(c - double(bf16_value(h))));
}

// per operator t: inv[t] = 2^-e with e such that max|C_t| 2^e lies in [2^14, 2^15)
__global__ void __launch_bounds__(kThreads) k_operator_scale(const double *C, int k, float *inv) {
    __shared__ double red[kThreads];
    const int t = blockIdx.x;
    double mx = 0.0;
    for (int64_t e = threadIdx.x; e < int64_t(k) * k; e += kThreads)
        mx = fmax(mx, fabs(C[int64_t(t) * k * k + e]));
    red[threadIdx.x] = mx;
    __syncthreads();
    for (int st = kThreads / 2; st > 0; st >>= 1) {
        if (threadIdx.x < st) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + st]);
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double m = red[0];
        // keep 2^-e a normal float; entries too small for fp16 then flush to 0
        // (operators below ~1e-38 contribute nothing at FP32 accuracy)
        const int e = m > 0.0 ? max(-126, min(126, 14 - ilogb(m))) : 0;
        inv[t] = float(ldexp(1.0, -e));
    }
}

__global__ void __launch_bounds__(kThreads)
k_cast_fp16(const double *C, int k, int kp, int batches, const float *inv, uint16_t *out) {
    const int64_t g = int64_t(blockIdx.x) * kThreads + threadIdx.x;
    const int64_t per = int64_t(kp) * kp;
    if (g >= per * batches) return;
    const int64_t b = g / per;
    const int i = int((g % per) / kp), j = int(g % kp);
    const double c = (i < k && j < k) ? C[b * k * k + int64_t(i) * k + j] : 0.0;
    const _Float16 h = static_cast<_Float16>(float(c / double(inv[b])));
    out[g] = __builtin_bit_cast(uint16_t, h);
}

inline int grid(int64_t n) { return int(ceil_div(n, kThreads)); }

int pad16(int k) { return int(ceil_div(k, 16) * 16); }

// eigen-decomposition of a Gram matrix -> sorted singular values, order, count
void gram_eig(DBuf<double> &G, DBuf<double> &Q, int m, double eps, DBuf<int32_t> &order,
              DBuf<double> &sv, int &count, hipStream_t s) {
    Q.alloc(int64_t(m) * m);
    k_identity<<<grid(int64_t(m) * m), kThreads, 0, s>>>(Q.p, m);
    BB_LAUNCH_CHECK();
    DBuf<int32_t> dsweeps(1), dcount(1);
    int wide_sweeps = -1;
    if (m >= kJacobiWideFrom) {
        wide_sweeps = jacobi_wide(G.p, Q.p, m, 60, 1e-14, s);
    } else {
        k_jacobi<<<1, kJacobiThreads, 0, s>>>(G.p, Q.p, m, 60, 1e-14, dsweeps.p);
        BB_LAUNCH_CHECK();
    }
    order.alloc(m);
    sv.alloc(m);
    BB_HIP(hipMemsetAsync(dcount.p, 0, sizeof(int32_t), s));
    k_eig_order<<<1, kThreads, 0, s>>>(G.p, m, eps, order.p, sv.p, dcount.p);
    BB_LAUNCH_CHECK();
    int32_t hc = 0, hs = 0;
    BB_HIP(hipMemcpyAsync(&hc, dcount.p, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    if (wide_sweeps < 0)
        BB_HIP(hipMemcpyAsync(&hs, dsweeps.p, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    BB_HIP(hipStreamSynchronize(s));
    if (wide_sweeps >= 0) hs = wide_sweeps;
    BB_INTERNAL(hs < 60, "Jacobi eigensolver did not converge");
    count = hc;
}

// C_t = sym * C_{315-t}^T for the upper half of the transfer vectors: the
// compact index of -t is 315 minus that of t (the 316 vectors sorted by an
// index that negation reverses)
__global__ void __launch_bounds__(kThreads)
k_mirror_operators(double *C, int k, double sym) {
    const int64_t g = int64_t(blockIdx.x) * kThreads + threadIdx.x;
    const int64_t half = int64_t(kNumT / 2) * k * k;
    if (g >= half) return;
    const int t = int(g / (int64_t(k) * k));
    const int ij = int(g % (int64_t(k) * k)), i = ij / k, j = ij % k;
    C[int64_t(kNumT - 1 - t) * k * k + int64_t(j) * k + i] = sym * C[g];
}

// Build one operator set from sampled K (316 x m x m, FP64).  sym: +1 for
// a symmetric kernel, -1 for a skew-symmetric one, 0 otherwise.  With
// symmetry K_{-t} = sym K_t^T (Section 2.5), so the thin matrix is the fat
// one transposed up to a permutation of blocks and a sign: its Gram matrix
// and singular values are the fat one's, V = U, and only the operators of
// the first 158 transfer vectors are formed; the rest are their (signed)
// transposes.
void compress_set(OpSet &set, DBuf<double> &K, int m, double eps, int sym, hipStream_t s) {
    if (eps == 0.0) {
        set.k = m;
        set.U64.alloc(int64_t(m) * m);
        set.V64.alloc(int64_t(m) * m);
        k_identity<<<grid(int64_t(m) * m), kThreads, 0, s>>>(set.U64.p, m);
        k_identity<<<grid(int64_t(m) * m), kThreads, 0, s>>>(set.V64.p, m);
        BB_LAUNCH_CHECK();
        set.C64 = std::move(K);
        return;
    }
    DBuf<double> Qf, Qt;
    DBuf<int32_t> of, ot;
    int kf = 0, kt = 0;
    {
        DBuf<double> Gf(int64_t(m) * m);
        GemmArgs g{m, m, m, kNumT, 1,
                   K.p, int64_t(m) * m, m, 1,          // A_b = K_t
                   K.p, int64_t(m) * m, 1, m,          // B_b = K_t^T
                   Gf.p, 0, m, 1};
        dgemm(g, s);
        gram_eig(Gf, Qf, m, eps, of, set.sv_fat, kf, s);
    }
    if (sym == 0) {
        DBuf<double> Gt(int64_t(m) * m);
        GemmArgs h{m, m, m, kNumT, 1,
                   K.p, int64_t(m) * m, 1, m,          // A_b = K_t^T
                   K.p, int64_t(m) * m, m, 1,          // B_b = K_t
                   Gt.p, 0, m, 1};
        dgemm(h, s);
        gram_eig(Gt, Qt, m, eps, ot, set.sv_thin, kt, s);
    } else {
        kt = kf;
        set.sv_thin.alloc(set.sv_fat.n);
        BB_HIP(hipMemcpyAsync(set.sv_thin.p, set.sv_fat.p, set.sv_fat.bytes(),
                              hipMemcpyDeviceToDevice, s));
    }
    const int k = std::max(std::max(kf, kt), 1);
    set.k = k;
    set.U64.alloc(int64_t(m) * k);
    set.V64.alloc(int64_t(m) * k);
    k_select_columns<<<grid(int64_t(m) * k), kThreads, 0, s>>>(Qf.p, m, of.p, k, set.U64.p);
    if (sym == 0)
        k_select_columns<<<grid(int64_t(m) * k), kThreads, 0, s>>>(Qt.p, m, ot.p, k, set.V64.p);
    else
        k_select_columns<<<grid(int64_t(m) * k), kThreads, 0, s>>>(Qf.p, m, of.p, k, set.V64.p);
    BB_LAUNCH_CHECK();
    // W_t = K_t V (m x k), C_t = U^T W_t (k x k)
    const int nt = sym == 0 ? kNumT : kNumT / 2;
    DBuf<double> W(int64_t(nt) * m * k);
    {
        GemmArgs g{m, k, m, nt, 0,
                   K.p, int64_t(m) * m, m, 1,
                   set.V64.p, 0, k, 1,
                   W.p, int64_t(m) * k, k, 1};
        dgemm(g, s);
    }
    set.C64.alloc(int64_t(kNumT) * k * k);
    {
        GemmArgs g{k, k, m, nt, 0,
                   set.U64.p, 0, 1, k,                 // A = U^T
                   W.p, int64_t(m) * k, k, 1,
                   set.C64.p, int64_t(k) * k, k, 1};
        dgemm(g, s);
    }
    if (sym != 0) {
        k_mirror_operators<<<grid(int64_t(kNumT / 2) * k * k), kThreads, 0, s>>>(set.C64.p, k,
                                                                                double(sym));
        BB_LAUNCH_CHECK();
    }
    BB_HIP(hipStreamSynchronize(s));
}

}  // namespace

void finalize_opset(OpSet &set, int m, int mp, int precision, hipStream_t s) {
    const int k = set.k;
    // MFMA K granularity: 16 for FP32 (16x16x4), 32 for the 16-bit paths (16x16x32)
    set.kp = precision == BBFMM_M2L_FP32 ? pad16(k) : int(ceil_div(k, 32) * 32);
    const int kp = set.kp;
    set.U32.alloc(int64_t(mp) * kp);
    set.VT32.alloc(int64_t(kp) * mp);
    k_cast_pad<<<grid(int64_t(mp) * kp), kThreads, 0, s>>>(set.U64.p, m, k, mp, kp, 1, set.U32.p);
    k_cast_pad_t<<<grid(int64_t(mp) * kp), kThreads, 0, s>>>(set.V64.p, m, k, mp, kp, set.VT32.p);
    const int64_t nc = int64_t(kNumT) * kp * kp;
    if (precision == BBFMM_M2L_FP32) {
        set.C32.alloc(nc);
        k_cast_pad<<<grid(nc), kThreads, 0, s>>>(set.C64.p, k, k, kp, kp, kNumT, set.C32.p);
    } else if (precision == BBFMM_M2L_BF16X3) {
        set.Chi.alloc(nc);
        set.Clo.alloc(nc);
        k_split_bf16<<<grid(nc), kThreads, 0, s>>>(set.C64.p, k, kp, kNumT, set.Chi.p, set.Clo.p);
    } else {
        set.C16.alloc(nc);
        set.Cinv.alloc(kNumT);
        k_operator_scale<<<kNumT, kThreads, 0, s>>>(set.C64.p, k, set.Cinv.p);
        k_cast_fp16<<<grid(nc), kThreads, 0, s>>>(set.C64.p, k, kp, kNumT, set.Cinv.p, set.C16.p);
    }
    BB_LAUNCH_CHECK();
    BB_HIP(hipStreamSynchronize(s));
}

void cheb_setup(bbfmm_ops *ops, hipStream_t s) {
    const int n = ops->n;
    const int len = 2 * kMaxOrder + 2 * kMaxOrder * kMaxOrder;
    DBuf<double> d(len);
    BB_HIP(hipMemsetAsync(d.p, 0, len * sizeof(double), s));
    k_cheb<<<1, 64, 0, s>>>(n, ops->nodes, d.p);
    BB_LAUNCH_CHECK();
    std::vector<double> h(len);
    BB_HIP(hipMemcpyAsync(h.data(), d.p, len * sizeof(double), hipMemcpyDeviceToHost, s));
    BB_HIP(hipStreamSynchronize(s));
    ChebConst &c = ops->cheb;
    c = ChebConst{};
    c.n = n;
    for (int i = 0; i < kMaxOrder; ++i) {
        c.s[i] = float(h[i]);
        c.w[i] = float(h[kMaxOrder + i]);
    }
    for (int o = 0; o < 2; ++o)
        for (int i = 0; i < kMaxOrder; ++i)
            for (int j = 0; j < kMaxOrder; ++j)
                c.T[o][i][j] = float(h[2 * kMaxOrder + (o * kMaxOrder + i) * kMaxOrder + j]);
}

void precompute_check(double eps, int precision) {
    BB_REQUIRE(std::isfinite(eps) && eps >= 0.0, "svd_eps must be finite and >= 0");
    // the singular values come from eigenvalues of Gram matrices (sigma^2),
    // which FP64 resolves down to about 1e-8 of the largest singular value:
    // a threshold below kMinSvdEps would cut inside round-off
    BB_REQUIRE(eps == 0.0 || eps >= kMinSvdEps || precision == BBFMM_M2L_FFT,
               "svd_eps must be 0 (no compression) or >= %g", kMinSvdEps);
    BB_REQUIRE(precision == BBFMM_M2L_FP32 || precision == BBFMM_M2L_BF16X3 ||
                   precision == BBFMM_M2L_FP16_SCALED || precision == BBFMM_M2L_FFT,
               "unsupported M2L precision %d", precision);
}

bbfmm_ops *precompute_impl(const bbfmm_tree *t, double eps, int precision, hipStream_t s) {
    precompute_check(eps, precision);
    BB_REQUIRE(t != nullptr, "tree is NULL");
    std::unique_ptr<bbfmm_ops> ops(new bbfmm_ops());
    ops->nodes = precision == BBFMM_M2L_FFT ? 1 : 0;
    ops->tree = t;
    ops->n = t->params.cheb_order;
    ops->m = ops->n * ops->n * ops->n;
    ops->mp = int(ceil_div(ops->m, 16) * 16);
    ops->precision = precision;
    ops->eps = eps;
    cheb_setup(ops.get(), s);
    const int L = t->leaf_level();
    if (L < 2) return ops.release();
    const int n = ops->n, m = ops->m;

    // Chebyshev nodes (FP64, first kMaxOrder entries) and transfer vectors
    DBuf<double> cheb(2 * kMaxOrder + 2 * kMaxOrder * kMaxOrder);
    BB_HIP(hipMemsetAsync(cheb.p, 0, cheb.bytes(), s));
    k_cheb<<<1, 64, 0, s>>>(n, ops->nodes, cheb.p);
    BB_LAUNCH_CHECK();
    const TransferTables &tt = transfer_tables();
    DBuf<int32_t> tvec(3 * kNumT);
    BB_HIP(hipMemcpyAsync(tvec.p, &tt.tvec[0][0], 3 * kNumT * sizeof(int32_t),
                          hipMemcpyHostToDevice, s));

    const int kid = t->params.kernel_id;
    const double a = t->params.kernel_param;
    auto sample = [&](double h) {
        DBuf<double> K(int64_t(kNumT) * m * m);
        k_sample<<<grid(int64_t(kNumT) * m * m), kThreads, 0, s>>>(kid, a, n, h, cheb.p, tvec.p,
                                                                    K.p);
        BB_LAUNCH_CHECK();
        return K;
    };
    // Section 2.5: symmetry (+1) or skew-symmetry (-1) of the kernel, and the
    // degree of a homogeneous one (0: not homogeneous)
    const int sym = (kid == BBFMM_K_INV_R || kid == BBFMM_K_EXP || kid == BBFMM_K_GAUSS) ? 1
                    : kid == BBFMM_K_DIPOLE_X ? -1 : 0;
    const int degree = kid == BBFMM_K_INV_R ? -1 : kid == BBFMM_K_DIPOLE_X ? -2 : 0;
    if (precision == BBFMM_M2L_FFT) {
        // equally spaced nodes: the uncompressed operators' spectra
        BB_REQUIRE(n >= 2, "the FFT M2L needs order >= 2");
        auto spectra = [&](double h) {
            std::unique_ptr<OpSet> set(new OpSet());
            set->k = m;
            set->kp = m;
            fft_operator_spectra(kid, a, n, h, tvec.p, set->Ghat, s);
            return set;
        };
        if (degree != 0) {
            std::unique_ptr<OpSet> set = spectra(1.0);
            for (int lvl = 2; lvl <= L; ++lvl) {
                ops->lv[lvl].set = set.get();
                ops->lv[lvl].scale = std::pow(t->half_width(lvl), double(degree));
            }
            ops->sets.push_back(std::move(set));
        } else {
            for (int lvl = 2; lvl <= L; ++lvl) {
                std::unique_ptr<OpSet> set = spectra(t->half_width(lvl));
                ops->lv[lvl].set = set.get();
                ops->lv[lvl].scale = 1.0;
                ops->sets.push_back(std::move(set));
            }
        }
    } else if (degree != 0) {
        // homogeneous: one set at h = 1, level factor h^degree
        std::unique_ptr<OpSet> set(new OpSet());
        DBuf<double> K = sample(1.0);
        compress_set(*set, K, m, eps, sym, s);
        finalize_opset(*set, m, ops->mp, precision, s);
        for (int lvl = 2; lvl <= L; ++lvl) {
            ops->lv[lvl].set = set.get();
            ops->lv[lvl].scale = std::pow(t->half_width(lvl), double(degree));
        }
        ops->sets.push_back(std::move(set));
    } else {
        for (int lvl = 2; lvl <= L; ++lvl) {
            std::unique_ptr<OpSet> set(new OpSet());
            DBuf<double> K = sample(t->half_width(lvl));
            compress_set(*set, K, m, eps, sym, s);
            finalize_opset(*set, m, ops->mp, precision, s);
            ops->lv[lvl].set = set.get();
            ops->lv[lvl].scale = 1.0;
            ops->sets.push_back(std::move(set));
        }
    }
    BB_HIP(hipStreamSynchronize(s));
    return ops.release();
}

}  // namespace bbfmm
