// k_order.hip -- spatial order of the grains for the row coefficients.
//
// The far-field test of the objective and gradient loops (a whole chunk of a
// wave below the skip threshold) pays only when the grains of a chunk (8 in the
// objective, a wave's 64 in the gradient) lie close together: then a pixel far
// from them is far from all of them.  A fit-form plan therefore stores the row
// coefficients of its grains in the Morton (Z-curve) order of their centroids;
// labels are mapped through the inverse permutation where the kernels meet them
// and the gradient is written back in the caller's grain order, so the order
// changes nothing but the rounding order of the sums over grains.
//
// Centroids come from exact integer sums (row, column, count per grain), so the
// order is deterministic.  Maps with more than PD_ORDER_MAX grains keep the
// identity order (the sort runs in one block's LDS).
#include "pd_host.h"

// Per grain: sum of columns, sum of rows, pixel count (int64 each).
// grid: (blocks over the largest map's pixels, n_maps); a wave takes 64
// consecutive pixels and adds each run of equal labels with one atomic per sum.
__global__ __launch_bounds__(PD_BLOCK) void k_order_sums(const MapDev *__restrict__ maps) {
  const MapDev &M = maps[blockIdx.y];
  if (M.order == nullptr) return;
  const long long n = (long long)M.H * M.W;
  const long long x = (long long)blockIdx.x * PD_BLOCK + threadIdx.x;
  const int lane = threadIdx.x % PD_WAVE;
  const bool valid = x < n;
  int g = -1;
  long long r = 0, c = 0;
  if (valid) {
    g = M.labels[x];
    if (g < 0 || g >= M.N) g = -1;
    r = x / M.W;
    c = x - r * M.W;
  }
  unsigned long long mask = __ballot(g >= 0);
  unsigned long long *sums = (unsigned long long *)M.order_sums;
  while (mask) {
    const int tgt = __builtin_amdgcn_readlane(g, __builtin_ctzll(mask));
    const bool mine = g == tgt;
    mask &= ~__ballot(mine);
    unsigned long long sc = mine ? (unsigned long long)c : 0ull;
    unsigned long long sr = mine ? (unsigned long long)r : 0ull;
    unsigned long long cnt = mine ? 1ull : 0ull;
    for (int o = PD_WAVE / 2; o > 0; o >>= 1) {
      sc += __shfl_xor(sc, o, PD_WAVE);
      sr += __shfl_xor(sr, o, PD_WAVE);
      cnt += __shfl_xor(cnt, o, PD_WAVE);
    }
    if (lane == 0) {
      atomicAdd(sums + (size_t)tgt, sc);
      atomicAdd(sums + (size_t)M.N + tgt, sr);
      atomicAdd(sums + 2 * (size_t)M.N + tgt, cnt);
    }
  }
}

__global__ __launch_bounds__(PD_BLOCK) void k_order_clear(const MapDev *__restrict__ maps) {
  const MapDev &M = maps[blockIdx.y];
  if (M.order == nullptr) return;
  const int i = blockIdx.x * PD_BLOCK + threadIdx.x;
  unsigned long long *sums = (unsigned long long *)M.order_sums;
  if (i < 3 * M.N) sums[i] = 0ull;
}

// Interleave the bits of two 16-bit integers (x in the even bits).
__device__ inline unsigned int morton2(unsigned int x, unsigned int y) {
  unsigned long long z = 0;
  for (int b = 0; b < 16; ++b) z |= (unsigned long long)(((x >> b) & 1u) << (2 * b)) |
                                   (unsigned long long)(((y >> b) & 1u) << (2 * b + 1));
  return (unsigned int)z;
}

// One block per map: keys (Morton code of the centroid, grain index) in LDS,
// bitonic sort, then order[j] and pos[order[j]] = j.  Empty grains go last.
constexpr int ORDER_THREADS = 1024;
__global__ __launch_bounds__(ORDER_THREADS) void k_order_sort(const MapDev *__restrict__ maps) {
  const MapDev &M = maps[blockIdx.x];
  if (M.order == nullptr) return;
  __shared__ unsigned long long key[PD_ORDER_MAX];
  const unsigned long long *sums = (const unsigned long long *)M.order_sums;
  int P2 = 1;
  while (P2 < M.N) P2 <<= 1;
  for (int i = threadIdx.x; i < P2; i += ORDER_THREADS) {
    unsigned long long k = ~0ull;
    if (i < M.N) {
      const unsigned long long cnt = sums[2 * (size_t)M.N + i];
      unsigned int code = 0xffffffffu;
      if (cnt > 0) {
        const unsigned long long cx = sums[i] / cnt, cy = sums[(size_t)M.N + i] / cnt;
        const unsigned int qx = (unsigned int)((cx * 65536ull) / (unsigned long long)M.W);
        const unsigned int qy = (unsigned int)((cy * 65536ull) / (unsigned long long)M.H);
        code = morton2(qx, qy);
      }
      k = ((unsigned long long)code << 32) | (unsigned int)i;
    }
    key[i] = k;
  }
  __syncthreads();
  for (int size = 2; size <= P2; size <<= 1) {
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      for (int t = threadIdx.x; t < P2 / 2; t += ORDER_THREADS) {
        const int lo = 2 * t - (t & (stride - 1));
        const int hi = lo + stride;
        const bool up = (lo & size) == 0;
        const unsigned long long a = key[lo], b = key[hi];
        if ((a > b) == up) {
          key[lo] = b;
          key[hi] = a;
        }
      }
      __syncthreads();
    }
  }
  int32_t *order = (int32_t *)M.order;
  int32_t *pos = (int32_t *)M.pos;
  for (int j = threadIdx.x; j < M.N; j += ORDER_THREADS) {
    const int i = (int)(unsigned int)(key[j] & 0xffffffffull);
    order[j] = i;
    pos[i] = j;
  }
}

void pd_launch_order(const MapDev *maps, int n_maps, long long max_px, int max_n, hipStream_t s) {
  if (n_maps <= 0) return;
  const unsigned bc = (unsigned)((3LL * max_n + PD_BLOCK - 1) / PD_BLOCK);
  k_order_clear<<<dim3(bc, n_maps), PD_BLOCK, 0, s>>>(maps);
  const unsigned bp = (unsigned)((max_px + PD_BLOCK - 1) / PD_BLOCK);
  if (bp > 0) k_order_sums<<<dim3(bp, n_maps), PD_BLOCK, 0, s>>>(maps);
  k_order_sort<<<n_maps, ORDER_THREADS, 0, s>>>(maps);
}
