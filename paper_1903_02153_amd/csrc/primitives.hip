// Device primitives used by the tree build: exclusive prefix sum and a
// stable LSD radix sort of (uint64 key, int32 value) pairs, plus the host
// tables of M2L transfer vectors.
//
// Both primitives are deterministic: the scan is a fixed tree of partial
// sums, the sort ranks equal digits by their position (wave ballots), so
// equal keys keep their input order -- the tie-break the octree needs.
#include "common.h"

namespace bbfmm {

// ------------------------------------------------------------ tables ----
TransferTables::TransferTables() {
    int c = 0;
    for (int tz = -3; tz <= 3; ++tz)
        for (int ty = -3; ty <= 3; ++ty)
            for (int tx = -3; tx <= 3; ++tx) {
                int a = tx < 0 ? -tx : tx, b = ty < 0 ? -ty : ty, d = tz < 0 ? -tz : tz;
                int mx = a > b ? a : b;
                mx = mx > d ? mx : d;
                if (mx < 2) continue;
                tvec[c][0] = tx; tvec[c][1] = ty; tvec[c][2] = tz;
                ++c;
            }
    for (int o = 0; o < 8; ++o) {
        int j = 0;
        for (int t = 0; t < kNumT; ++t) {
            t_slot[o][t] = -1;
            bool ok = true;
            for (int d = 0; d < 3; ++d) {
                // target coordinate 2P + b: parents adjacent iff -2-b <= t <= 3-b
                int b = (o >> d) & 1;
                if (tvec[t][d] < -2 - b || tvec[t][d] > 3 - b) ok = false;
            }
            if (ok) { slot_t[o][j] = t; t_slot[o][t] = j; ++j; }
        }
    }
}

const TransferTables &transfer_tables() {
    static TransferTables tables;
    return tables;
}

// -------------------------------------------------------------- scan ----
namespace {

constexpr int kScanThreads = 256;
constexpr int kScanItems = 4;
constexpr int kScanTile = kScanThreads * kScanItems;

__device__ inline int wave_incl_scan(int v, int lane) {
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        int t = __shfl_up(v, d, 64);
        if (lane >= d) v += t;
    }
    return v;
}

__global__ void __launch_bounds__(kScanThreads)
k_scan_tile(const int32_t *in, int32_t *out, int32_t *sums, int64_t n) {
    __shared__ int wsum[kScanThreads / 64];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int64_t base = int64_t(blockIdx.x) * kScanTile + int64_t(tid) * kScanItems;
    int v[kScanItems];
    int tot = 0;
#pragma unroll
    for (int i = 0; i < kScanItems; ++i) {
        v[i] = (base + i < n) ? in[base + i] : 0;
        tot += v[i];
    }
    int inc = wave_incl_scan(tot, lane);
    if (lane == 63) wsum[w] = inc;
    __syncthreads();
    int woff = 0;
    for (int j = 0; j < w; ++j) woff += wsum[j];
    int run = woff + inc - tot;
#pragma unroll
    for (int i = 0; i < kScanItems; ++i) {
        if (base + i < n) out[base + i] = run;
        run += v[i];
    }
    if (tid == kScanThreads - 1 && sums) sums[blockIdx.x] = woff + inc;
}

__global__ void __launch_bounds__(kScanThreads)
k_scan_add(int32_t *out, const int32_t *offs, int64_t n) {
    const int32_t add = offs[blockIdx.x];
    const int64_t base = int64_t(blockIdx.x) * kScanTile;
    for (int i = threadIdx.x; i < kScanTile; i += kScanThreads)
        if (base + i < n) out[base + i] += add;
}

void scan_rec(const int32_t *in, int32_t *out, int64_t n, hipStream_t s, int32_t *total_dev) {
    const int64_t nb = ceil_div(n, kScanTile);
    if (nb == 1) {
        k_scan_tile<<<1, kScanThreads, 0, s>>>(in, out, total_dev, n);
        BB_LAUNCH_CHECK();
        return;
    }
    DBuf<int32_t> sums(nb);
    k_scan_tile<<<nb, kScanThreads, 0, s>>>(in, out, sums.p, n);
    BB_LAUNCH_CHECK();
    scan_rec(sums.p, sums.p, nb, s, total_dev);
    k_scan_add<<<nb, kScanThreads, 0, s>>>(out, sums.p, n);
    BB_LAUNCH_CHECK();
    // sums must outlive the kernels that read it
    BB_HIP(hipStreamSynchronize(s));
}

}  // namespace

int64_t scan_exclusive(const int32_t *in, int32_t *out, int64_t n, hipStream_t s) {
    if (n <= 0) return 0;
    DBuf<int32_t> total(1);
    scan_rec(in, out, n, s, total.p);
    int32_t h = 0;
    BB_HIP(hipMemcpyAsync(&h, total.p, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    BB_HIP(hipStreamSynchronize(s));
    return h;
}

// -------------------------------------------------------- radix sort ----
namespace {

constexpr int kRsThreads = 256;
constexpr int kRsItems = 8;
constexpr int kRsTile = kRsThreads * kRsItems;
constexpr int kRsRadix = 256;

__global__ void __launch_bounds__(kRsThreads)
k_radix_count(const uint64_t *keys, int64_t n, int shift, int32_t *hist, int nblocks) {
    __shared__ int cnt[kRsRadix];
    const int tid = threadIdx.x;
    cnt[tid] = 0;
    __syncthreads();
    const int64_t base = int64_t(blockIdx.x) * kRsTile;
    for (int it = 0; it < kRsItems; ++it) {
        int64_t idx = base + it * kRsThreads + tid;
        if (idx < n) atomicAdd(&cnt[(keys[idx] >> shift) & 255], 1);
    }
    __syncthreads();
    hist[int64_t(tid) * nblocks + blockIdx.x] = cnt[tid];
}

__global__ void __launch_bounds__(kRsThreads)
k_radix_scatter(const uint64_t *kin, const int32_t *vin, uint64_t *kout, int32_t *vout,
                int64_t n, int shift, const int32_t *offs, int nblocks) {
    __shared__ int run[kRsRadix];
    __shared__ int wcnt[kRsThreads / 64][kRsRadix];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    run[tid] = offs[int64_t(tid) * nblocks + blockIdx.x];
    for (int ww = 0; ww < kRsThreads / 64; ++ww) wcnt[ww][tid] = 0;
    __syncthreads();
    const int64_t base = int64_t(blockIdx.x) * kRsTile;
    const uint64_t lt = (1ull << lane) - 1ull;
    for (int it = 0; it < kRsItems; ++it) {
        const int64_t idx = base + it * kRsThreads + tid;
        const bool valid = idx < n;
        uint64_t key = valid ? kin[idx] : 0ull;
        int32_t val = valid ? vin[idx] : 0;
        const int d = int((key >> shift) & 255);
        // lanes of this wave holding the same (valid, digit)
        uint64_t peers;
        {
            uint64_t m = __ballot(valid);
            peers = valid ? m : ~m;
        }
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const int bit = (d >> b) & 1;
            uint64_t m = __ballot(bit);
            peers &= bit ? m : ~m;
        }
        const int rank = __popcll(peers & lt);
        const int leader = __builtin_ctzll(peers);
        if (valid && lane == leader) wcnt[w][d] = __popcll(peers);
        __syncthreads();
        if (valid) {
            int off = 0;
            for (int ww = 0; ww < w; ++ww) off += wcnt[ww][d];
            const int pos = run[d] + off + rank;
            kout[pos] = key;
            vout[pos] = val;
        }
        __syncthreads();
        int t = 0;
        for (int ww = 0; ww < kRsThreads / 64; ++ww) {
            t += wcnt[ww][tid];
            wcnt[ww][tid] = 0;
        }
        run[tid] += t;
        __syncthreads();
    }
}

}  // namespace

void radix_sort_pairs(uint64_t *keys, int32_t *vals, int64_t n, int bits, hipStream_t s) {
    if (n <= 1 || bits <= 0) return;
    const int nb = int(ceil_div(n, kRsTile));
    DBuf<uint64_t> k2(n);
    DBuf<int32_t> v2(n);
    DBuf<int32_t> hist(int64_t(kRsRadix) * nb);
    uint64_t *ka = keys, *kb = k2.p;
    int32_t *va = vals, *vb = v2.p;
    for (int shift = 0; shift < bits; shift += 8) {
        k_radix_count<<<nb, kRsThreads, 0, s>>>(ka, n, shift, hist.p, nb);
        BB_LAUNCH_CHECK();
        scan_exclusive(hist.p, hist.p, int64_t(kRsRadix) * nb, s);
        k_radix_scatter<<<nb, kRsThreads, 0, s>>>(ka, va, kb, vb, n, shift, hist.p, nb);
        BB_LAUNCH_CHECK();
        std::swap(ka, kb);
        std::swap(va, vb);
    }
    if (ka != keys) {
        BB_HIP(hipMemcpyAsync(keys, ka, n * sizeof(uint64_t), hipMemcpyDeviceToDevice, s));
        BB_HIP(hipMemcpyAsync(vals, va, n * sizeof(int32_t), hipMemcpyDeviceToDevice, s));
    }
    BB_HIP(hipStreamSynchronize(s));
}

}  // namespace bbfmm
