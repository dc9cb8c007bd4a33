// Particle re-sort by containing tet with compaction: a stable LSD radix
// sort of (key = tet, or n_tets for a free slot; value = slot index) with
// 6-bit digits, then a gather of every particle array into scratch and a
// copy back.  Stable ranking comes from each thread owning a contiguous
// run of items: per-thread digit counts, a per-digit prefix over threads in
// LDS, and a prefix over blocks from one scan kernel -- no atomics, so the
// order (and everything computed after it) is deterministic.
#include "common.h"
#include "sort.h"

namespace fp {

namespace {

constexpr int kBins = 64;  // 6-bit digits
constexpr int kThreads = 256;
constexpr int kPer = 16;   // items per thread
constexpr int kTile = kThreads * kPer;

// counts[b][t] of the digits of thread t's items (b < kBins)
__device__ inline void thread_counts(const uint32_t* key, int64_t n,
                                     int64_t base, int shift,
                                     uint16_t (*cnt)[kThreads]) {
  for (int b = 0; b < kBins; ++b) cnt[b][threadIdx.x] = 0;
  const int64_t i0 = base + (int64_t)threadIdx.x * kPer;
  for (int k = 0; k < kPer; ++k) {
    const int64_t i = i0 + k;
    if (i < n) cnt[(key[i] >> shift) & (kBins - 1)][threadIdx.x] += 1;
  }
}

}  // namespace

__global__ void __launch_bounds__(kThreads) k_sort_keys(SortArgs a) {
  const int64_t n = *a.n_slots;
  if (blockIdx.x == 0 && threadIdx.x == 0) *a.n_live = 0;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int32_t t = a.tet[i];
    a.key[0][i] = t < 0 ? (uint32_t)a.n_tets : (uint32_t)t;
    a.val[0][i] = (uint32_t)i;
  }
}

// Per-block digit totals: hist[bin * nblocks + block].
__global__ void __launch_bounds__(kThreads) k_sort_hist(SortArgs a, int src,
                                                        int shift) {
  __shared__ uint16_t cnt[kBins][kThreads];
  const int64_t n = *a.n_slots;
  const int64_t base = (int64_t)blockIdx.x * kTile;
  thread_counts(a.key[src], n, base, shift, cnt);
  __syncthreads();
  if (threadIdx.x < kBins) {
    uint32_t s = 0;
    for (int t = 0; t < kThreads; ++t) s += cnt[threadIdx.x][t];
    a.hist[(int64_t)threadIdx.x * gridDim.x + blockIdx.x] = s;
  }
}

// Exclusive scan of hist (bin-major) in one block: every wave owns 4 bins;
// it sums their per-block counts, the 64 bin totals are scanned in LDS, and
// each wave then rescans its bins (64 counts at a time, shuffle scan) from
// the bin's offset.
// The counts of a bin's run of kScanRun blocks are loaded into registers
// before any arithmetic, so the loads of a wave are in flight together.
constexpr int kScanRun = 16 * 64;

__global__ void __launch_bounds__(1024) k_sort_scan(SortArgs a, int nblocks) {
  __shared__ uint32_t bin_total[kBins];
  __shared__ uint32_t bin_off[kBins];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int nwaves = blockDim.x >> 6;
  for (int b = wave; b < kBins; b += nwaves) {
    uint32_t s = 0;
    for (int j0 = 0; j0 < nblocks; j0 += kScanRun) {
      uint32_t v[16];
#pragma unroll
      for (int k = 0; k < 16; ++k) {
        const int j = j0 + k * 64 + lane;
        v[k] = j < nblocks ? a.hist[(int64_t)b * nblocks + j] : 0u;
      }
#pragma unroll
      for (int k = 0; k < 16; ++k) s += v[k];
    }
    for (int off = 32; off >= 1; off >>= 1) s += __shfl_xor(s, off, 64);
    if (lane == 0) bin_total[b] = s;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t run = 0;
    for (int b = 0; b < kBins; ++b) {
      bin_off[b] = run;
      run += bin_total[b];
    }
  }
  __syncthreads();
  for (int b = wave; b < kBins; b += nwaves) {
    uint32_t carry = bin_off[b];
    for (int j0 = 0; j0 < nblocks; j0 += kScanRun) {
      uint32_t v[16];
#pragma unroll
      for (int k = 0; k < 16; ++k) {
        const int j = j0 + k * 64 + lane;
        v[k] = j < nblocks ? a.hist[(int64_t)b * nblocks + j] : 0u;
      }
#pragma unroll
      for (int k = 0; k < 16; ++k) {
        const int j = j0 + k * 64 + lane;
        uint32_t inc = v[k];
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
          const uint32_t o = __shfl_up(inc, off, 64);
          if (lane >= off) inc += o;
        }
        if (j < nblocks) a.hist[(int64_t)b * nblocks + j] = carry + inc - v[k];
        carry += __shfl(inc, 63, 64);
      }
    }
  }
}

__global__ void __launch_bounds__(kThreads) k_sort_scatter(SortArgs a, int src,
                                                           int shift) {
  __shared__ uint16_t cnt[kBins][kThreads];
  __shared__ uint32_t pre[kBins][kThreads];
  const int64_t n = *a.n_slots;
  const int64_t base = (int64_t)blockIdx.x * kTile;
  const uint32_t* key = a.key[src];
  const uint32_t* val = a.val[src];
  thread_counts(key, n, base, shift, cnt);
  __syncthreads();
  // per-bin exclusive prefix over threads: 4 threads per bin, 64 each
  {
    const int b = threadIdx.x >> 2, q = threadIdx.x & 3;
    uint32_t s = 0;
    for (int t = q * 64; t < q * 64 + 64; ++t) {
      pre[b][t] = s;
      s += cnt[b][t];
    }
    // combine the 4 quarter sums (in LDS order, deterministic)
    __shared__ uint32_t qs[kBins][4];
    qs[b][q] = s;
    __syncthreads();
    uint32_t add = 0;
    for (int k = 0; k < q; ++k) add += qs[b][k];
    for (int t = q * 64; t < q * 64 + 64; ++t) pre[b][t] += add;
  }
  __syncthreads();
  const int64_t i0 = base + (int64_t)threadIdx.x * kPer;
  for (int k = 0; k < kPer; ++k) {
    const int64_t i = i0 + k;
    if (i >= n) break;
    const uint32_t kk = key[i];
    const int b = (kk >> shift) & (kBins - 1);
    const uint32_t pos = a.hist[(int64_t)b * gridDim.x + blockIdx.x] +
                         pre[b][threadIdx.x];
    pre[b][threadIdx.x] += 1;
    a.key[src ^ 1][pos] = kk;
    a.val[src ^ 1][pos] = val[i];
  }
}

// Gather every particle array into scratch in sorted order; the last live
// position sets the new slot count.
__global__ void __launch_bounds__(kThreads) k_sort_gather(SortArgs a, int src) {
  const int64_t n = *a.n_slots;
  const uint32_t* key = a.key[src];
  const uint32_t* val = a.val[src];
  for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < n;
       j += (int64_t)gridDim.x * blockDim.x) {
    const bool live = key[j] < (uint32_t)a.n_tets;
    const bool last = live && (j + 1 == n || key[j + 1] >= (uint32_t)a.n_tets);
    if (last) *a.n_live = (int32_t)(j + 1);
    if (j == 0 && !live) *a.n_live = 0;
    if (!live) continue;
    const int64_t s = val[j];
    if (a.real_bytes == 8) {
      for (int f = 0; f < 6; ++f)
        reinterpret_cast<double*>(a.s_real[f])[j] = reinterpret_cast<const double*>(a.real[f])[s];
    } else {
      for (int f = 0; f < 6; ++f)
        reinterpret_cast<float*>(a.s_real[f])[j] = reinterpret_cast<const float*>(a.real[f])[s];
    }
    a.s_w[j] = a.w[s];
    a.s_tet[j] = a.tet[s];
    a.s_birth[j] = a.birth[s];
    a.s_id[j] = a.id[s];
  }
}

__global__ void __launch_bounds__(kThreads) k_sort_copyback(SortArgs a) {
  const int64_t n = *a.n_live;
  for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < n;
       j += (int64_t)gridDim.x * blockDim.x) {
    if (a.real_bytes == 8) {
      for (int f = 0; f < 6; ++f)
        reinterpret_cast<double*>(a.real[f])[j] = reinterpret_cast<const double*>(a.s_real[f])[j];
    } else {
      for (int f = 0; f < 6; ++f)
        reinterpret_cast<float*>(a.real[f])[j] = reinterpret_cast<const float*>(a.s_real[f])[j];
    }
    a.w[j] = a.s_w[j];
    a.tet[j] = a.s_tet[j];
    a.birth[j] = a.s_birth[j];
    a.id[j] = a.s_id[j];
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    *a.n_slots = (int32_t)n;
    if (a.stats) a.stats->n_slots = n;
  }
}

hipError_t sort_particles(const SortArgs& a, int64_t capacity, int n_cu,
                          hipStream_t s) {
  const int nblocks = (int)((capacity + kTile - 1) / kTile);
  const int grid = n_cu * 4;
  hipLaunchKernelGGL(k_sort_keys, dim3(grid), dim3(kThreads), 0, s, a);
  int bits = 1;
  while ((1ll << bits) <= a.n_tets) ++bits;
  int src = 0;
  for (int shift = 0; shift < bits; shift += 6) {
    hipLaunchKernelGGL(k_sort_hist, dim3(nblocks), dim3(kThreads), 0, s, a, src, shift);
    hipLaunchKernelGGL(k_sort_scan, dim3(1), dim3(1024), 0, s, a, nblocks);
    hipLaunchKernelGGL(k_sort_scatter, dim3(nblocks), dim3(kThreads), 0, s, a, src, shift);
    src ^= 1;
  }
  hipLaunchKernelGGL(k_sort_gather, dim3(grid), dim3(kThreads), 0, s, a, src);
  hipLaunchKernelGGL(k_sort_copyback, dim3(grid), dim3(kThreads), 0, s, a);
  return hipGetLastError();
}

size_t sort_scratch_bytes(int64_t capacity, int real_bytes) {
  const int64_t nblocks = (capacity + kTile - 1) / kTile;
  return (size_t)capacity * (16 + 6 * (size_t)real_bytes + 8 + 4 + 4 + 8) +
         (size_t)kBins * nblocks * 4 + 4096;
}

}  // namespace fp
