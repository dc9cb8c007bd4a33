// Particle re-sort by containing tet with compaction: a stable LSD radix
// sort of (key = tet, or n_tets for a free slot; value = slot index) with
// 8-bit digits, then a gather of every particle array into scratch and a
// copy back.
//
// One pass over a digit is three launches:
//   k_sort_hist     digit counts of every tile of kSortTile items;
//   k_sort_scan     one workgroup per digit: exclusive scan of that digit's
//                   counts over the tiles, and the digit's total;
//   k_sort_scatter  every wave ranks the 64 items of a round among the
//                   lanes with the same digit (eight ballots; lanes are in
//                   item order, so the rank is stable), per-wave digit
//                   counters in LDS carry the rank across rounds and waves,
//                   the tile is reordered by digit in LDS and written out in
//                   runs that are contiguous in the destination.
// No atomic operation decides an order, so the permutation (and everything
// computed after it) is deterministic.
#include "common.h"
#include "sort.h"

namespace fp {

namespace {

constexpr int kBins = kSortBins;
constexpr int kThreads = 256;
constexpr int kWaves = kThreads / 64;
constexpr int kRounds = kSortTile / kThreads;  // rounds of 64 items per wave
static_assert(kThreads == kBins, "one thread per digit in the tile sums");
static_assert(kSortTile == kWaves * kRounds * 64, "tile = waves x rounds x 64");

// Exclusive prefix of v over the threads of the workgroup (thread order);
// *total receives the sum.  Every thread must call it.
__device__ inline uint32_t block_exscan(uint32_t v, uint32_t* wsum,
                                        uint32_t* total) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  uint32_t inc = v;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const uint32_t o = __shfl_up(inc, off, 64);
    if (lane >= off) inc += o;
  }
  if (lane == 63) wsum[wave] = inc;
  __syncthreads();
  uint32_t before = 0, all = 0;
#pragma unroll
  for (int w = 0; w < kWaves; ++w) {
    if (w < wave) before += wsum[w];
    all += wsum[w];
  }
  __syncthreads();
  *total = all;
  return before + inc - v;
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

// Digit counts of tile b: hist[digit * ntiles + b].  (Integer counts: the
// order of the LDS additions does not matter.)
__global__ void __launch_bounds__(kThreads) k_sort_hist(SortArgs a, int src,
                                                        int shift) {
  __shared__ uint32_t cnt[kBins];
  const int64_t n = *a.n_slots;
  cnt[threadIdx.x] = 0;
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * kSortTile;
  const uint32_t* key = a.key[src];
  for (int k = threadIdx.x; k < kSortTile; k += kThreads) {
    const int64_t i = base + k;
    if (i < n) atomicAdd(&cnt[(key[i] >> shift) & (kBins - 1)], 1u);
  }
  __syncthreads();
  a.hist[(int64_t)threadIdx.x * gridDim.x + blockIdx.x] = cnt[threadIdx.x];
}

// Workgroup d: exclusive scan of hist[d][0..ntiles) in place, total[d].
__global__ void __launch_bounds__(kThreads) k_sort_scan(SortArgs a,
                                                        int ntiles) {
  __shared__ uint32_t wsum[kWaves];
  uint32_t* row = a.hist + (int64_t)blockIdx.x * ntiles;
  uint32_t carry = 0;
  for (int j0 = 0; j0 < ntiles; j0 += kThreads) {
    const int j = j0 + threadIdx.x;
    const uint32_t v = j < ntiles ? row[j] : 0u;
    uint32_t chunk;
    const uint32_t ex = block_exscan(v, wsum, &chunk);
    if (j < ntiles) row[j] = carry + ex;
    carry += chunk;
  }
  if (threadIdx.x == 0) a.total[blockIdx.x] = carry;
}

__global__ void __launch_bounds__(kThreads) k_sort_scatter(SortArgs a, int src,
                                                           int shift) {
  __shared__ uint32_t wc[kWaves][kBins];  // per-wave digit counts, then bases
  __shared__ uint32_t tstart[kBins];      // first slot of a digit in the tile
  __shared__ uint32_t gbase[kBins];       // destination of that slot
  __shared__ uint32_t s_key[kSortTile];
  __shared__ uint32_t s_val[kSortTile];
  __shared__ uint32_t wsum[kWaves];
  const int64_t n = *a.n_slots;
  const int64_t base = (int64_t)blockIdx.x * kSortTile;
  if (base >= n) return;  // the whole workgroup: no barrier is skipped
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int w = 0; w < kWaves; ++w) wc[w][threadIdx.x] = 0;
  __syncthreads();
  const uint32_t* key = a.key[src];
  const uint32_t* val = a.val[src];
  // wave w owns items [w, w + 1) * kRounds * 64 of the tile, round r the
  // 64 items from r * 64 on: lane order is item order
  const int64_t w0 = base + (int64_t)wave * kRounds * 64 + lane;
  uint32_t kr[kRounds], vr[kRounds], rk[kRounds];
#pragma unroll
  for (int r = 0; r < kRounds; ++r) {
    const int64_t i = w0 + r * 64;
    kr[r] = i < n ? key[i] : 0u;
    vr[r] = i < n ? val[i] : 0u;
  }
  const uint64_t below_me = (1ull << lane) - 1ull;
#pragma unroll
  for (int r = 0; r < kRounds; ++r) {
    const bool ok = w0 + r * 64 < n;
    const uint32_t d = (kr[r] >> shift) & (kBins - 1);
    // lanes holding an item with the same digit as this lane
    uint64_t peers = __ballot(ok);
#pragma unroll
    for (int bit = 0; bit < 8; ++bit) {
      const bool one = (d >> bit) & 1u;
      const uint64_t m = __ballot(one);
      peers &= one ? m : ~m;
    }
    const uint32_t prev = wc[wave][d];
    rk[r] = prev + (uint32_t)__popcll(peers & below_me);
    // the highest lane of each digit group advances the wave's counter
    // (after every lane of the wave has read it: LDS keeps a wave's order)
    if (ok && (peers >> lane) == 1ull)
      wc[wave][d] = prev + (uint32_t)__popcll(peers);
  }
  __syncthreads();
  {
    // thread b: the digit's wave bases inside the tile, its first slot in
    // the tile and the destination of that slot
    const int b = threadIdx.x;
    uint32_t cnt = 0;
#pragma unroll
    for (int w = 0; w < kWaves; ++w) {
      const uint32_t c = wc[w][b];
      wc[w][b] = cnt;
      cnt += c;
    }
    uint32_t all;
    const uint32_t ts = block_exscan(cnt, wsum, &all);
    const uint32_t bb = block_exscan(a.total[b], wsum, &all);
    tstart[b] = ts;
    gbase[b] = bb + a.hist[(int64_t)b * gridDim.x + blockIdx.x];
  }
  __syncthreads();
#pragma unroll
  for (int r = 0; r < kRounds; ++r) {
    if (w0 + r * 64 >= n) continue;
    const uint32_t d = (kr[r] >> shift) & (kBins - 1);
    const uint32_t p = tstart[d] + wc[wave][d] + rk[r];
    s_key[p] = kr[r];
    s_val[p] = vr[r];
  }
  __syncthreads();
  const int m = n - base < kSortTile ? (int)(n - base) : kSortTile;
  uint32_t* okey = a.key[src ^ 1];
  uint32_t* oval = a.val[src ^ 1];
  for (int j = threadIdx.x; j < m; j += kThreads) {
    const uint32_t kk = s_key[j];
    const uint32_t d = (kk >> shift) & (kBins - 1);
    const uint32_t pos = gbase[d] + ((uint32_t)j - tstart[d]);
    okey[pos] = kk;
    oval[pos] = s_val[j];
  }
}

// Gather every particle array into scratch in sorted order; the last live
// position sets the new slot count.  The sorted order is close to the
// previous one, so the sources of a run of outputs lie in a narrow window:
// each XCD (block index mod 8) takes one contiguous eighth of the outputs,
// so that a source line is fetched into one XCD's L2 rather than into
// every XCD whose blocks interleave over it.
__global__ void __launch_bounds__(kThreads) k_sort_gather(SortArgs a, int src) {
  const int64_t n = *a.n_slots;
  const uint32_t* key = a.key[src];
  const uint32_t* val = a.val[src];
  const int parts = gridDim.x % 8 == 0 ? 8 : 1;
  const int part = (int)blockIdx.x % parts;
  const int64_t per_part = (n + parts - 1) / parts;
  const int64_t lo = part * per_part;
  const int64_t hi = lo + per_part < n ? lo + per_part : n;
  const int64_t stride = (int64_t)(gridDim.x / parts) * blockDim.x;
  for (int64_t j = lo + (int64_t)(blockIdx.x / parts) * blockDim.x + threadIdx.x;
       j < hi; j += stride) {
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

// The slot count of a re-sort whose output stays in the scratch arrays.
__global__ void k_sort_count(SortArgs a) {
  if (threadIdx.x != 0) return;
  const int32_t n = *a.n_live;
  *a.n_slots = n;
  if (a.stats) a.stats->n_slots = n;
}

__global__ void __launch_bounds__(kThreads) k_particles_copy(SortArgs a) {
  const int64_t n = *a.n_slots;
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
}

int sort_tiles(int64_t capacity) {
  return (int)((capacity + kSortTile - 1) / kSortTile);
}

hipError_t sort_particles(const SortArgs& a, int64_t capacity, int n_cu,
                          hipStream_t s, bool copyback) {
  const int ntiles = sort_tiles(capacity);
  const int grid = n_cu * 4;
  hipLaunchKernelGGL(k_sort_keys, dim3(grid), dim3(kThreads), 0, s, a);
  int bits = 1;
  while ((1ll << bits) <= a.n_tets) ++bits;
  int src = 0;
  for (int shift = 0; shift < bits; shift += 8) {
    hipLaunchKernelGGL(k_sort_hist, dim3(ntiles), dim3(kThreads), 0, s, a, src, shift);
    hipLaunchKernelGGL(k_sort_scan, dim3(kBins), dim3(kThreads), 0, s, a, ntiles);
    hipLaunchKernelGGL(k_sort_scatter, dim3(ntiles), dim3(kThreads), 0, s, a, src, shift);
    src ^= 1;
  }
  hipLaunchKernelGGL(k_sort_gather, dim3(grid), dim3(kThreads), 0, s, a, src);
  if (copyback)
    hipLaunchKernelGGL(k_sort_copyback, dim3(grid), dim3(kThreads), 0, s, a);
  else
    hipLaunchKernelGGL(k_sort_count, dim3(1), dim3(64), 0, s, a);
  return hipGetLastError();
}

hipError_t copy_particles(const SortArgs& a, int n_cu, hipStream_t s) {
  hipLaunchKernelGGL(k_particles_copy, dim3(n_cu * 4), dim3(kThreads), 0, s, a);
  return hipGetLastError();
}

size_t sort_scratch_bytes(int64_t capacity, int real_bytes) {
  const int64_t ntiles = sort_tiles(capacity);
  return (size_t)capacity * (16 + 6 * (size_t)real_bytes + 8 + 4 + 4 + 8) +
         (size_t)kBins * ntiles * 4 + kBins * 4 + 8192;
}

}  // namespace fp
