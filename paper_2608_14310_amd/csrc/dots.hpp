// Partial dot products of several vectors with one vector, shared by the
// host-driven and the graph-captured FGMRES so that both reduce in the same
// order (Section 5 CGS2 inner products).
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

namespace cav {
// part[i * nblk + blk] = sum over this block's elements of V_i . w.
// Each block owns a contiguous chunk; thread t of the block takes elements
// s + t, s + t + TPB, ... and sums them in that order, then a shuffle tree
// per wavefront and the wavefronts in order. The chunk's loads for one
// vector are issued together (DOT_EPT per thread, w kept in registers when
// the chunk is one tile), and the wavefront sums of up to DOT_G vectors are
// combined after one barrier.
constexpr int DOT_EPT = 8;
constexpr int DOT_G = 32;
template <int TPB>
__device__ __forceinline__ void dots_block(const double* __restrict__ V, int64_t ldv, int k,
                                           const double* __restrict__ w, int64_t n, double* __restrict__ part,
                                           int nblk) {
  __shared__ double sh[DOT_G][TPB / 64];
  const int64_t chunk = (n + nblk - 1) / nblk;
  const int64_t s = int64_t(blockIdx.x) * chunk, e = min(n, s + chunk);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  constexpr int64_t TILE = int64_t(TPB) * DOT_EPT;
  const bool one_tile = chunk <= TILE;
  double wr[DOT_EPT];
#pragma unroll
  for (int u = 0; u < DOT_EPT; ++u) {
    const int64_t t = s + threadIdx.x + int64_t(u) * TPB;
    wr[u] = (one_tile && t < e) ? w[t] : 0.0;
  }
  for (int g0 = 0; g0 < k; g0 += DOT_G) {
    const int gk = min(DOT_G, k - g0);
    for (int gi = 0; gi < gk; ++gi) {
      const double* vi = V + int64_t(g0 + gi) * ldv;
      double acc = 0.0;
      if (one_tile) {
        double v[DOT_EPT];
#pragma unroll
        for (int u = 0; u < DOT_EPT; ++u) {
          const int64_t t = s + threadIdx.x + int64_t(u) * TPB;
          v[u] = t < e ? vi[t] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < DOT_EPT; ++u)
          if (s + threadIdx.x + int64_t(u) * TPB < e) acc += v[u] * wr[u];
      } else {
        for (int64_t t = s + threadIdx.x; t < e; t += TPB) acc += vi[t] * w[t];
      }
      for (int o = 32; o > 0; o >>= 1) acc += __shfl_down(acc, o, 64);
      if (lane == 0) sh[gi][wid] = acc;
    }
    __syncthreads();
    if (int(threadIdx.x) < gk) {
      double r = 0.0;
      for (int q = 0; q < TPB / 64; ++q) r += sh[threadIdx.x][q];
      part[int64_t(g0 + threadIdx.x) * nblk + blockIdx.x] = r;
    }
    __syncthreads();
  }
}

}  // namespace cav
