// k_assign.hip -- hard arg-min assignment F_theta and accuracy (Section 2.1,
// 2.2): the launch over all row segments (the per-block work is assign_block in
// assign_dev.h), the fixed-order count reduction and label validation.
#include "assign_dev.h"

template <int DMAX>
__global__ __launch_bounds__(PD_BLOCK) void k_assign(const MapDev *__restrict__ maps,
                                                     const int32_t *__restrict__ off, int n_maps,
                                                     int total) {
  constexpr int KM = (DMAX + 1) * (DMAX + 2) / 2;
  __shared__ double sth[AS_CHUNK * KM];
  const int item0 = blockIdx.x * PD_WAVES_PER_BLOCK;
  if (item0 >= total) return;
  const int m = pd_find_map(off, n_maps, item0);
  const MapDev &M = maps[m];
  if (PD_GATED(M)) return;
  PD_DISPATCH_UPTO(DMAX, M.d, (assign_block<D>(M, item0 - off[m], sth)));
}

// One block per map: fixed-order sum of the per-wave correct counts.
__global__ __launch_bounds__(PD_BLOCK) void k_reduce_count(const MapDev *__restrict__ maps) {
  const MapDev &M = maps[blockIdx.x];
  if (M.n_correct == nullptr || PD_GATED(M)) return;
  __shared__ long long red[PD_BLOCK];
  long long s = 0;
  for (int t = threadIdx.x; t < M.a_items / PD_WAVES_PER_BLOCK; t += PD_BLOCK) s += M.part_c[t];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = PD_BLOCK / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) *M.n_correct = red[0];
}

// bad[m] = 1 if some label of map m lies outside [0, N).  grid: (blocks, n_maps).
__global__ __launch_bounds__(PD_BLOCK) void k_validate(const MapDev *__restrict__ maps,
                                                       int32_t *bad) {
  const MapDev &M = maps[blockIdx.y];
  const long long n = (long long)M.H * M.W;
  int b = 0;
  for (long long j = (long long)blockIdx.x * PD_BLOCK + threadIdx.x; j < n;
       j += (long long)gridDim.x * PD_BLOCK) {
    const int g = M.labels[j];
    b |= (g < 0 || g >= M.N);
  }
  if (b) bad[blockIdx.y] = 1;
}

// The canonical arg-min of the pixels that the certified objective launch could
// not decide (unc_list), counted into fb_count.  grid: (blocks, n_maps); the
// blocks stride over the list 256 pixels at a time.
template <int DMAX>
__global__ __launch_bounds__(PD_BLOCK) void k_assign_list(const MapDev *__restrict__ maps) {
  constexpr int KM = (DMAX + 1) * (DMAX + 2) / 2;
  __shared__ double sth[AS_CHUNK * KM];
  __shared__ int bsum;
  const MapDev &M = maps[blockIdx.y];
  if (M.cert == nullptr || PD_GATED(M)) return;
  const int cap = M.rows * M.W;
  const int count = min(*pd_uni(M.unc_count), cap);
  for (int base = blockIdx.x * PD_BLOCK; base < count; base += gridDim.x * PD_BLOCK) {
    const int q = base + (int)threadIdx.x;
    const bool valid = q < count;
    const int pix = valid ? pd_glb(M.unc_list)[q] : M.row0 * M.W;
    const int r = pix / M.W, c = pix - r * M.W;
    bool bad = false;
    int best = 0;
    PD_DISPATCH_UPTO(DMAX, M.d, (best = canonical_argmin<D, false>(M, r, c, sth, &bad)));
    const int ok = (valid && !bad && best == pd_glb(M.labels)[pix]) ? 1 : 0;
    if (threadIdx.x == 0) bsum = 0;
    __syncthreads();
    const long long ws = pd_wave_sum_i64(ok);
    if ((threadIdx.x % PD_WAVE) == 0 && ws) atomicAdd(&bsum, (int)ws);
    __syncthreads();
    if (threadIdx.x == 0 && bsum) atomicAdd((unsigned long long *)M.fb_count, (unsigned long long)bsum);
  }
}

void pd_launch_assign_list(int dmax, const MapDev *maps, int n_maps, hipStream_t s) {
  const dim3 grid(256, n_maps);
  switch (dmax) {
    case 2: k_assign_list<2><<<grid, PD_BLOCK, 0, s>>>(maps); break;
    case 4: k_assign_list<4><<<grid, PD_BLOCK, 0, s>>>(maps); break;
    case 6: k_assign_list<6><<<grid, PD_BLOCK, 0, s>>>(maps); break;
    default: k_assign_list<8><<<grid, PD_BLOCK, 0, s>>>(maps); break;
  }
}

void pd_launch_assign(int dmax, const MapDev *maps, const int32_t *off, int n_maps, int total,
                      bool count, hipStream_t s) {
  const int blocks = (total + PD_WAVES_PER_BLOCK - 1) / PD_WAVES_PER_BLOCK;
  switch (dmax) {
    case 2: k_assign<2><<<blocks, PD_BLOCK, 0, s>>>(maps, off, n_maps, total); break;
    case 4: k_assign<4><<<blocks, PD_BLOCK, 0, s>>>(maps, off, n_maps, total); break;
    case 6: k_assign<6><<<blocks, PD_BLOCK, 0, s>>>(maps, off, n_maps, total); break;
    default: k_assign<8><<<blocks, PD_BLOCK, 0, s>>>(maps, off, n_maps, total); break;
  }
  if (count) k_reduce_count<<<n_maps, PD_BLOCK, 0, s>>>(maps);
}

void pd_launch_validate(const MapDev *maps, int n_maps, int32_t *bad, hipStream_t s) {
  k_validate<<<dim3(64, n_maps), PD_BLOCK, 0, s>>>(maps, bad);
}
