// fit.hip -- fitter scratch, the longest-first ordering kernel and the launch
// of the persistent fit kernel.
#include "fit_impl.hpp"

namespace hf {

namespace {

constexpr int kMaxRankB = 1 << 16;

// Rank every histogram by size, longest first, ties by index: a strict total
// order, so the ranks form a permutation.  O(B^2) comparisons staged through
// LDS tiles; used for B <= kMaxRankB.

__global__ __launch_bounds__(kBlock) void k_rank_sizes(const int64_t* __restrict__ offsets, int B,
                                                      int32_t* __restrict__ order) {
  __shared__ int64_t tile[kBlock];
  const int b = blockIdx.x * kBlock + threadIdx.x;
  const int64_t mine = b < B ? offsets[b + 1] - offsets[b] : 0;
  int rank = 0;
  for (int j0 = 0; j0 < B; j0 += kBlock) {
    const int j = j0 + threadIdx.x;
    tile[threadIdx.x] = j < B ? offsets[j + 1] - offsets[j] : 0;
    __syncthreads();
    const int lim = min(kBlock, B - j0);
    for (int q = 0; q < lim; ++q) {
      const int64_t o = tile[q];
      rank += (o > mine) || (o == mine && j0 + q < b);
    }
    __syncthreads();
  }
  if (b < B) order[rank] = b;
}

// Batches of at most kSortB histograms are ordered by one block instead: a
// bitonic sort in LDS of 64-bit keys (the size's complement above the
// index, so ascending keys are sizes descending, then indices ascending:
// the same permutation).  Measured on 4096 histograms: 58 us, against
// 253 us for the comparison count above (on 16 blocks).
constexpr int kSortB = 4096;
constexpr int kSortThreads = 1024;

__global__ __launch_bounds__(kSortThreads) void k_sort_sizes(const int64_t* __restrict__ offsets,
                                                             int B, int32_t* __restrict__ order) {
  __shared__ uint64_t key[kSortB];
  constexpr uint64_t kSizeMax = (uint64_t(1) << 48) - 1;  // sizes above compare as equal
  int n = 1;
  while (n < B) n <<= 1;
  for (int i = threadIdx.x; i < n; i += kSortThreads) {
    uint64_t k = ~uint64_t(0);
    if (i < B) {
      const int64_t sz = offsets[i + 1] - offsets[i];
      const uint64_t c = sz <= 0 ? 0 : (static_cast<uint64_t>(sz) > kSizeMax ? kSizeMax : sz);
      k = ((kSizeMax - c) << 16) | static_cast<uint64_t>(i);
    }
    key[i] = k;
  }
  __syncthreads();
  for (int k = 2; k <= n; k <<= 1) {
    for (int j = k >> 1; j > 0; j >>= 1) {
      for (int i = threadIdx.x; i < n; i += kSortThreads) {
        const int p = i ^ j;
        if (p > i) {
          const uint64_t x = key[i], y = key[p];
          if ((x > y) == ((i & k) == 0)) {
            key[i] = y;
            key[p] = x;
          }
        }
      }
      __syncthreads();
    }
  }
  for (int i = threadIdx.x; i < B; i += kSortThreads)
    order[i] = static_cast<int32_t>(key[i] & 0xffffu);
}

FitLaunchFn pick_fit(int ng, int bkg, int obj, int blk) {
  switch (ng) {
    case 0:
      return pick_fit_ng0(bkg, obj, blk);
    case 1:
      return pick_fit_ng1(bkg, obj, blk);
    case 2:
      return pick_fit_ng2(bkg, obj, blk);
    case 3:
      return pick_fit_ng3(bkg, obj, blk);
    case 4:
      return pick_fit_ng4(bkg, obj, blk);
    default:
      return nullptr;
  }
}

}  // namespace

// The ordering buffer is allocated once, for the largest batch that is
// ranked (kMaxRankB histograms, 256 KiB), so no fit_batch call allocates,
// frees or synchronises, and a graph captured earlier keeps a valid pointer.
hipError_t fit_scratch_init(FitScratch* s) {
  hipError_t e = hipMalloc(&s->counters, 256);
  if (e != hipSuccess) return e;
  e = hipMalloc(&s->order, sizeof(int32_t) * static_cast<size_t>(kMaxRankB));
  if (e != hipSuccess) return e;
  s->cap = kMaxRankB;
  return hipMemset(s->counters, 0, 256);
}

void fit_scratch_free(FitScratch* s) {
  if (s->order) (void)hipFree(s->order);
  if (s->counters) (void)hipFree(s->counters);
  s->order = nullptr;
  s->counters = nullptr;
  s->cap = 0;
}

int fit_max_cache_bins(int n_gauss, int bkg, int obj, int block) {
  FitLaunchFn fn = pick_fit(n_gauss, bkg, obj, block);
  int m = 0;
  if (!fn || fn(FitArgs{}, 0, nullptr, &m) != hipSuccess) return 0;
  return m > 0 ? m : 0;
}

int fit_max_wave_bins(int n_gauss, int bkg, int obj, int block) {
  FitLaunchFn fn = pick_fit(n_gauss, bkg, obj, block);
  int m = 0;
  if (!fn || fn(FitArgs{}, -1, nullptr, &m) != hipSuccess) return 0;
  return m > 0 ? m : 0;
}

hipError_t launch_fit(int n_gauss, int bkg, FitArgs a, int num_cu, FitScratch* s, hipStream_t st) {
  FitLaunchFn fn = pick_fit(n_gauss, bkg, a.obj, s->block);
  if (!fn) return hipErrorNotSupported;
  a.cache_bins = s->cache_bins;
  a.wave_bins = s->wave_bins;
  // batches above kMaxRankB run in index order (no ranking pass)
  a.sorted = (a.B <= kMaxRankB && a.B <= s->cap) ? 1 : 0;
  a.order = s->order;
  a.counters = s->counters;
  if (a.sorted && a.B <= kSortB) {
    hipLaunchKernelGGL(k_sort_sizes, dim3(1), dim3(kSortThreads), 0, st, a.offsets, a.B, a.order);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  } else if (a.sorted) {
    hipLaunchKernelGGL(k_rank_sizes, dim3((a.B + kBlock - 1) / kBlock), dim3(kBlock), 0, st,
                       a.offsets, a.B, a.order);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  int grid = num_cu * s->wg_per_cu;
  if (grid > a.B) grid = a.B;
  return fn(a, grid, st, nullptr);
}

}  // namespace hf
