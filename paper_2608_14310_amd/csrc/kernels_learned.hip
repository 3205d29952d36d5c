// Learned correction stage: a small periodic conv net on the grid's (u, v, p)
// channels, its training kernels (forward, loss, backward, Adam) and the C ABI
// of the net handle.
//
// The net N: R^{3 x N x N} -> R^{3 x N x N} is
//   y1 = W1 * x, a1 = relu(y1); y2 = W2 * a1, a2 = relu(y2); y3 = W3 * a2,
// with 3x3 periodic cross-correlations, 3 -> 32 -> 32 -> 3 channels and no
// biases. Pixel (i, j) holds u_ij, v_ij and p_ij. Weights, the input and the
// hidden activations are bfloat16 (round to nearest even from FP32); every sum
// accumulates in FP32. Layer 2 (a dense 288 -> 32 contraction per pixel) runs
// on the matrix cores (16x16x16 bf16 MFMA); layers 1 and 3, the backward
// convolutions and the weight gradients are FP32 vector code. Hidden
// activations are NHWC (32 channels per pixel, contiguous), inputs and outputs
// are planar [b][channel][i][j] like the solver's vectors.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>

#include "cav_internal.hpp"

namespace cav {

namespace {
constexpr int TPB = 256;

__device__ __host__ inline uint16_t f2bf(float f) {
  uint32_t u;
  memcpy(&u, &f, 4);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return uint16_t(u >> 16);
}
__device__ inline float bf2f(uint16_t b) { return __uint_as_float(uint32_t(b) << 16); }
__device__ inline float bfround(float f) { return bf2f(f2bf(f)); }
__device__ inline uint32_t pack2(float lo, float hi) {
  return uint32_t(f2bf(lo)) | (uint32_t(f2bf(hi)) << 16);
}

// master weights -> bf16-rounded kernel layouts
__global__ void k_pack(const float* __restrict__ w, float* __restrict__ pk, uint16_t* __restrict__ w2m) {
  const int t = blockIdx.x * TPB + threadIdx.x;
  if (t >= NET_W) return;
  const uint16_t hb = f2bf(w[t]);
  const float v = bf2f(hb);
  if (t < 864) {
    const int co = t / 27, ci = (t / 9) % 3, a = (t / 3) % 3, c = t % 3;
    pk[PK_L1F + ((a * 3 + c) * 3 + ci) * 32 + co] = v;
  } else if (t < 864 + 9216) {
    const int u = t - 864;
    const int co = u / 288, ci = (u / 9) % 32, a = (u / 3) % 3, c = u % 3;
    pk[PK_L2T + ((a * 3 + c) * 32 + co) * 32 + ci] = v;
    w2m[co * 288 + (a * 3 + c) * 32 + ci] = hb;
  } else {
    const int u = t - 864 - 9216;
    const int co = u / 288, ci = (u / 9) % 32, a = (u / 3) % 3, c = u % 3;
    pk[PK_L3F + ((a * 3 + c) * 32 + ci) * 3 + co] = v;
    pk[PK_L3T + ((a * 3 + c) * 3 + co) * 32 + ci] = v;
  }
}

template <typename T>
__device__ inline float in_value(T x, double scale);
template <>
__device__ inline float in_value<float>(float x, double) { return bfround(x); }
template <>
__device__ inline float in_value<double>(double x, double scale) { return bfround(float(x * scale)); }

// Layer 1 (3 -> 32, VALU): one pixel per thread. Input planar (sample idx[b]
// or b); for FP64 input each sample is scaled by 1/sqrt(nrm2[b]) first.
template <typename T>
__global__ __launch_bounds__(TPB) void k_l1(const T* __restrict__ in, const int32_t* __restrict__ idx,
                                             const double* __restrict__ nrm2, int lgN,
                                             const float* __restrict__ w1f, uint16_t* __restrict__ a1) {
  __shared__ float w[864];
  for (int t = threadIdx.x; t < 864; t += TPB) w[t] = w1f[t];
  __syncthreads();
  const int N = 1 << lgN, msk = N - 1;
  const int64_t n2 = int64_t(N) * N;
  const int64_t p = int64_t(blockIdx.x) * TPB + threadIdx.x;
  if (p >= n2) return;
  const int b = blockIdx.y;
  const int64_t sb = idx ? idx[b] : b;
  const T* x = in + sb * 3 * n2;
  double scale = 1.0;
  if (nrm2) {
    const double q = nrm2[b];
    scale = q > 0.0 ? 1.0 / sqrt(q) : 0.0;
  }
  const int i = int(p >> lgN), j = int(p & msk);
  float acc[32];
#pragma unroll
  for (int co = 0; co < 32; ++co) acc[co] = 0.f;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const int64_t row = int64_t((i + a - 1) & msk) << lgN;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const int64_t q = row + ((j + c - 1) & msk);
#pragma unroll
      for (int ci = 0; ci < 3; ++ci) {
        const float v = in_value<T>(x[ci * n2 + q], scale);
        const float* wr = &w[((a * 3 + c) * 3 + ci) * 32];
#pragma unroll
        for (int co = 0; co < 32; ++co) acc[co] = fmaf(wr[co], v, acc[co]);
      }
    }
  }
  uint4* dst = reinterpret_cast<uint4*>(a1 + ((int64_t(b) * n2 + p) << 5));
#pragma unroll
  for (int h = 0; h < 4; ++h) {
    uint4 o;
    o.x = pack2(fmaxf(acc[8 * h + 0], 0.f), fmaxf(acc[8 * h + 1], 0.f));
    o.y = pack2(fmaxf(acc[8 * h + 2], 0.f), fmaxf(acc[8 * h + 3], 0.f));
    o.z = pack2(fmaxf(acc[8 * h + 4], 0.f), fmaxf(acc[8 * h + 5], 0.f));
    o.w = pack2(fmaxf(acc[8 * h + 6], 0.f), fmaxf(acc[8 * h + 7], 0.f));
    dst[h] = o;
  }
}

// Layer 2 (32 -> 32) on the matrix cores. Per pixel the layer is a 288-long
// contraction, k = (a*3 + c)*32 + ci. A workgroup owns an 8 x 32 pixel tile of
// one sample; its 10 x 34 halo tile of a1 is staged in LDS (pixel stride 40
// bf16 to spread LDS banks). Each wave owns two rows = four 16-pixel strips and
// both 16-channel output blocks: D[co][pix] = sum_k W[co][k] B[k][pix] with
// v_mfma_f32_16x16x16_bf16 (A: lane l holds row l%16, k 4(l/16)..+3; B: column
// l%16, the same k; D: lane l holds rows 4(l/16)..+3 of column l%16).
typedef short v4s __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));
constexpr int L2_TH = 8, L2_TW = 32, L2_PS = 40;
constexpr int L2_HW = L2_TW + 2, L2_HP = (L2_TH + 2) * L2_HW;

__global__ __launch_bounds__(TPB) void k_l2(const uint16_t* __restrict__ a1, int lgN,
                                             const uint16_t* __restrict__ w2m, uint16_t* __restrict__ a2) {
  __shared__ __align__(16) uint16_t tile[L2_HP * L2_PS];
  const int N = 1 << lgN, msk = N - 1;
  const int64_t n2 = int64_t(N) * N;
  const int j0 = blockIdx.x * L2_TW, i0 = blockIdx.y * L2_TH, b = blockIdx.z;
  const uint16_t* src = a1 + int64_t(b) * n2 * 32;
  for (int t = threadIdx.x; t < L2_HP * 4; t += TPB) {
    const int px = t >> 2, ch = t & 3;
    const int r = px / L2_HW, cc = px - r * L2_HW;
    const int ii = (i0 - 1 + r) & msk, jj = (j0 - 1 + cc) & msk;
    const uint4 v = *reinterpret_cast<const uint4*>(src + ((int64_t(ii) << lgN) + jj) * 32 + ch * 8);
    *reinterpret_cast<uint4*>(&tile[px * L2_PS + ch * 8]) = v;
  }
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int lr = lane & 15, lg = lane >> 4;
  v4s A0[18], A1[18];
#pragma unroll
  for (int s = 0; s < 18; ++s) {
    A0[s] = *reinterpret_cast<const v4s*>(w2m + lr * 288 + 16 * s + 4 * lg);
    A1[s] = *reinterpret_cast<const v4s*>(w2m + (16 + lr) * 288 + 16 * s + 4 * lg);
  }
  __syncthreads();
  v4f acc[4][2];
#pragma unroll
  for (int st = 0; st < 4; ++st) acc[st][0] = acc[st][1] = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int s = 0; s < 18; ++s) {
    const int ac = s >> 1, a = ac / 3, c = ac % 3, ci0 = 16 * (s & 1) + 4 * lg;
#pragma unroll
    for (int st = 0; st < 4; ++st) {
      const int r = 2 * wv + (st >> 1), js = st & 1;
      const int px = (r + a) * L2_HW + 16 * js + lr + c;
      const v4s B = *reinterpret_cast<const v4s*>(&tile[px * L2_PS + ci0]);
      acc[st][0] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(A0[s], B, acc[st][0], 0, 0, 0);
      acc[st][1] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(A1[s], B, acc[st][1], 0, 0, 0);
    }
  }
#pragma unroll
  for (int st = 0; st < 4; ++st) {
    const int i = i0 + 2 * wv + (st >> 1), j = j0 + 16 * (st & 1) + lr;
    if (i >= N || j >= N) continue;
    uint16_t* dst = a2 + ((int64_t(b) * n2 + (int64_t(i) << lgN) + j) << 5);
#pragma unroll
    for (int mb = 0; mb < 2; ++mb) {
      const v4f d = acc[st][mb];
      uint2 o;
      o.x = pack2(fmaxf(d[0], 0.f), fmaxf(d[1], 0.f));
      o.y = pack2(fmaxf(d[2], 0.f), fmaxf(d[3], 0.f));
      *reinterpret_cast<uint2*>(dst + 16 * mb + 4 * lg) = o;
    }
  }
}

// Layer 3 (32 -> 3, VALU): one pixel per thread. FP32 output, or FP64 output
// scaled by sqrt(nrm2[b]).
template <typename TO>
__global__ __launch_bounds__(TPB) void k_l3(const uint16_t* __restrict__ a2, int lgN, const float* __restrict__ w3f,
                                             const double* __restrict__ nrm2, TO* __restrict__ out) {
  __shared__ float w[864];
  for (int t = threadIdx.x; t < 864; t += TPB) w[t] = w3f[t];
  __syncthreads();
  const int N = 1 << lgN, msk = N - 1;
  const int64_t n2 = int64_t(N) * N;
  const int64_t p = int64_t(blockIdx.x) * TPB + threadIdx.x;
  if (p >= n2) return;
  const int b = blockIdx.y;
  const int i = int(p >> lgN), j = int(p & msk);
  float acc0 = 0.f, acc1 = 0.f, acc2 = 0.f;
  for (int a = 0; a < 3; ++a) {
    const int64_t row = int64_t((i + a - 1) & msk) << lgN;
    for (int c = 0; c < 3; ++c) {
      const int64_t q = row + ((j + c - 1) & msk);
      const uint4* sp = reinterpret_cast<const uint4*>(a2 + ((int64_t(b) * n2 + q) << 5));
#pragma unroll
      for (int h = 0; h < 4; ++h) {
        const uint4 v = sp[h];
        const uint32_t wd[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          const float x = bf2f(uint16_t(wd[e >> 1] >> (16 * (e & 1))));
          const float* wr = &w[((a * 3 + c) * 32 + 8 * h + e) * 3];
          acc0 = fmaf(wr[0], x, acc0);
          acc1 = fmaf(wr[1], x, acc1);
          acc2 = fmaf(wr[2], x, acc2);
        }
      }
    }
  }
  TO* o = out + int64_t(b) * 3 * n2 + p;
  if constexpr (sizeof(TO) == 8) {
    const double sc = nrm2 ? sqrt(nrm2[b]) : 1.0;
    o[0] = double(acc0) * sc;
    o[n2] = double(acc1) * sc;
    o[2 * n2] = double(acc2) * sc;
  } else {
    o[0] = acc0;
    o[n2] = acc1;
    o[2 * n2] = acc2;
  }
}

// ---- backward ----
// g2 = (W3^T * g3) masked by a2 > 0. One pixel per thread; NHWC FP32 output.
__global__ __launch_bounds__(TPB) void k_l3_bwd(const float* __restrict__ g3, const uint16_t* __restrict__ a2,
                                                 int lgN, const float* __restrict__ w3t, float* __restrict__ g2) {
  __shared__ float w[864];
  for (int t = threadIdx.x; t < 864; t += TPB) w[t] = w3t[t];
  __syncthreads();
  const int N = 1 << lgN, msk = N - 1;
  const int64_t n2 = int64_t(N) * N;
  const int64_t p = int64_t(blockIdx.x) * TPB + threadIdx.x;
  if (p >= n2) return;
  const int b = blockIdx.y;
  const int i = int(p >> lgN), j = int(p & msk);
  float acc[32];
#pragma unroll
  for (int ci = 0; ci < 32; ++ci) acc[ci] = 0.f;
  const float* gb = g3 + int64_t(b) * 3 * n2;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const int64_t row = int64_t((i - a + 1) & msk) << lgN;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const int64_t q = row + ((j - c + 1) & msk);
#pragma unroll
      for (int co = 0; co < 3; ++co) {
        const float gv = gb[co * n2 + q];
        const float* wr = &w[((a * 3 + c) * 3 + co) * 32];
#pragma unroll
        for (int ci = 0; ci < 32; ++ci) acc[ci] = fmaf(wr[ci], gv, acc[ci]);
      }
    }
  }
  const int64_t o = (int64_t(b) * n2 + p) << 5;
  const uint4* ap = reinterpret_cast<const uint4*>(a2 + o);
  float4* dst = reinterpret_cast<float4*>(g2 + o);
#pragma unroll
  for (int h = 0; h < 4; ++h) {
    const uint4 v = ap[h];
    const uint32_t wd[4] = {v.x, v.y, v.z, v.w};
    float m[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) m[e] = ((wd[e >> 1] >> (16 * (e & 1))) & 0xFFFFu) != 0 ? 1.f : 0.f;
    dst[2 * h] = make_float4(acc[8 * h] * m[0], acc[8 * h + 1] * m[1], acc[8 * h + 2] * m[2], acc[8 * h + 3] * m[3]);
    dst[2 * h + 1] =
        make_float4(acc[8 * h + 4] * m[4], acc[8 * h + 5] * m[5], acc[8 * h + 6] * m[6], acc[8 * h + 7] * m[7]);
  }
}

// g1 = (W2^T * g2) masked by a1 > 0. One pixel per thread; weights in LDS.
__global__ __launch_bounds__(TPB) void k_l2_bwd(const float* __restrict__ g2, const uint16_t* __restrict__ a1,
                                                 int lgN, const float* __restrict__ w2t, float* __restrict__ g1) {
  __shared__ float w[9216];
  for (int t = threadIdx.x; t < 9216; t += TPB) w[t] = w2t[t];
  __syncthreads();
  const int N = 1 << lgN, msk = N - 1;
  const int64_t n2 = int64_t(N) * N;
  const int64_t p = int64_t(blockIdx.x) * TPB + threadIdx.x;
  if (p >= n2) return;
  const int b = blockIdx.y;
  const int i = int(p >> lgN), j = int(p & msk);
  float acc[32];
#pragma unroll
  for (int ci = 0; ci < 32; ++ci) acc[ci] = 0.f;
  for (int a = 0; a < 3; ++a) {
    const int64_t row = int64_t((i - a + 1) & msk) << lgN;
    for (int c = 0; c < 3; ++c) {
      const int64_t q = row + ((j - c + 1) & msk);
      const float4* sp = reinterpret_cast<const float4*>(g2 + ((int64_t(b) * n2 + q) << 5));
      for (int h = 0; h < 8; ++h) {
        const float4 gv4 = sp[h];
        const float gvs[4] = {gv4.x, gv4.y, gv4.z, gv4.w};
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const float* wr = &w[((a * 3 + c) * 32 + 4 * h + e) * 32];
#pragma unroll
          for (int ci = 0; ci < 32; ++ci) acc[ci] = fmaf(wr[ci], gvs[e], acc[ci]);
        }
      }
    }
  }
  const int64_t o = (int64_t(b) * n2 + p) << 5;
  const uint4* ap = reinterpret_cast<const uint4*>(a1 + o);
  float4* dst = reinterpret_cast<float4*>(g1 + o);
#pragma unroll
  for (int h = 0; h < 4; ++h) {
    const uint4 v = ap[h];
    const uint32_t wd[4] = {v.x, v.y, v.z, v.w};
    float m[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) m[e] = ((wd[e >> 1] >> (16 * (e & 1))) & 0xFFFFu) != 0 ? 1.f : 0.f;
    dst[2 * h] = make_float4(acc[8 * h] * m[0], acc[8 * h + 1] * m[1], acc[8 * h + 2] * m[2], acc[8 * h + 3] * m[3]);
    dst[2 * h + 1] =
        make_float4(acc[8 * h + 4] * m[4], acc[8 * h + 5] * m[5], acc[8 * h + 6] * m[6], acc[8 * h + 7] * m[7]);
  }
}

// Weight gradients dW[co][ci][a][c] = sum_pix g[co][pix] x[ci][pix + (a-1, c-1)].
// KIND 3: g = g3 (planar), x = a2; KIND 2: g = g2 (NHWC), x = a1; KIND 1: g = g1
// (NHWC), x = bf16(input) (planar, sample idx[b]). A workgroup walks 8 x 8 pixel
// tiles (tile = blockIdx.x + k gridDim.x), staging g and the 10 x 10 halo of x
// in LDS; each thread owns a 4 (co) x 4 (ci) block of one tap (a, c) and
// writes its partial sums for the reduction kernel.
template <int KIND>
struct WG {
  static constexpr int CO = KIND == 3 ? 3 : 32, CI = KIND == 1 ? 3 : 32;
  static constexpr int CO4 = (CO + 3) / 4, CI4 = (CI + 3) / 4;
  static constexpr int NT = 9 * CO4 * CI4;
  static constexpr int BS = (NT + 63) / 64 * 64;
  static constexpr int NWL = CO * CI * 9;
};

template <int KIND>
__global__ __launch_bounds__(WG<KIND>::BS) void k_wgrad(const float* __restrict__ g, const void* __restrict__ xsrc,
                                                         const int32_t* __restrict__ idx, int lgN, int B,
                                                         float* __restrict__ part) {
  using P = WG<KIND>;
  constexpr int GW = P::CO4 * 4, XW = P::CI4 * 4;
  __shared__ __align__(16) float gs[64 * GW];
  __shared__ __align__(16) float xs[100 * XW];
  const int N = 1 << lgN, msk = N - 1;
  const int64_t n2 = int64_t(N) * N;
  const int tps = (N >> 3) * (N >> 3);
  const int ntiles = B * tps;
  const int t = threadIdx.x;
  const int ac = t / (P::CO4 * P::CI4), cob = (t / P::CI4) % P::CO4, cib = t % P::CI4;
  const int a = ac / 3, c = ac % 3;
  float acc[4][4];
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int v = 0; v < 4; ++v) acc[u][v] = 0.f;
  for (int tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const int b = tile / tps, tt = tile - b * tps;
    const int i0 = (tt / (N >> 3)) * 8, j0 = (tt % (N >> 3)) * 8;
    __syncthreads();
    for (int e = t; e < 64 * GW; e += P::BS) {
      const int px = e / GW, co = e - px * GW;
      const int64_t q = (int64_t(i0 + (px >> 3)) << lgN) + j0 + (px & 7);
      float v = 0.f;
      if (co < P::CO) {
        if constexpr (KIND == 3)
          v = g[(int64_t(b) * 3 + co) * n2 + q];
        else
          v = g[((int64_t(b) * n2 + q) << 5) + co];
      }
      gs[e] = v;
    }
    for (int e = t; e < 100 * XW; e += P::BS) {
      const int hp = e / XW, ci = e - hp * XW;
      const int ii = (i0 - 1 + hp / 10) & msk, jj = (j0 - 1 + hp % 10) & msk;
      const int64_t q = (int64_t(ii) << lgN) + jj;
      float v = 0.f;
      if (ci < P::CI) {
        if constexpr (KIND == 1) {
          const float* in = static_cast<const float*>(xsrc);
          const int64_t sb = idx ? idx[b] : b;
          v = bfround(in[(sb * 3 + ci) * n2 + q]);
        } else {
          const uint16_t* xa = static_cast<const uint16_t*>(xsrc);
          v = bf2f(xa[((int64_t(b) * n2 + q) << 5) + ci]);
        }
      }
      xs[e] = v;
    }
    __syncthreads();
    if (t < P::NT) {
      for (int p = 0; p < 64; ++p) {
        const int pi = p >> 3, pj = p & 7;
        const float4 gv = *reinterpret_cast<const float4*>(&gs[p * GW + cob * 4]);
        const float4 xv = *reinterpret_cast<const float4*>(&xs[((pi + a) * 10 + pj + c) * XW + cib * 4]);
        const float gg[4] = {gv.x, gv.y, gv.z, gv.w}, xx[4] = {xv.x, xv.y, xv.z, xv.w};
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
          for (int v = 0; v < 4; ++v) acc[u][v] = fmaf(gg[u], xx[v], acc[u][v]);
      }
    }
  }
  if (t < P::NT) {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int co = cob * 4 + u;
      if (co >= P::CO) continue;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int ci = cib * 4 + v;
        if (ci >= P::CI) continue;
        part[int64_t(blockIdx.x) * P::NWL + ((co * P::CI + ci) * 3 + a) * 3 + c] = acc[u][v];
      }
    }
  }
}

__global__ void k_wgrad_reduce(const float* __restrict__ part, int nblk, int nwl, float* __restrict__ grad) {
  const int w = blockIdx.x * TPB + threadIdx.x;
  if (w >= nwl) return;
  float s = 0.f;
  for (int k = 0; k < nblk; ++k) s += part[int64_t(k) * nwl + w];
  grad[w] = s;
}

// Loss sums per sample in FP64: se = ||e_b||^2, sd = ||y3_b - e_b||^2.
__device__ inline void block_pair_sum(double& a, double& b, double* sh) {
  sh[threadIdx.x] = a;
  sh[TPB + threadIdx.x] = b;
  __syncthreads();
  for (int s = TPB / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) {
      sh[threadIdx.x] += sh[threadIdx.x + s];
      sh[TPB + threadIdx.x] += sh[TPB + threadIdx.x + s];
    }
    __syncthreads();
  }
  a = sh[0];
  b = sh[TPB];
}

__global__ __launch_bounds__(TPB) void k_loss_partial(const float* __restrict__ y3, const float* __restrict__ eh,
                                                       const int32_t* __restrict__ idx, int64_t n3,
                                                       double* __restrict__ part) {
  __shared__ double sh[2 * TPB];
  const int b = blockIdx.y;
  const int64_t sb = idx ? idx[b] : b;
  double se = 0.0, sd = 0.0;
  for (int64_t k = int64_t(blockIdx.x) * TPB + threadIdx.x; k < n3; k += int64_t(gridDim.x) * TPB) {
    const double e = eh[sb * n3 + k], y = y3[int64_t(b) * n3 + k];
    se += e * e;
    sd += (y - e) * (y - e);
  }
  block_pair_sum(se, sd, sh);
  if (threadIdx.x == 0) {
    part[(int64_t(b) * gridDim.x + blockIdx.x) * 2] = se;
    part[(int64_t(b) * gridDim.x + blockIdx.x) * 2 + 1] = sd;
  }
}

__global__ void k_loss_final(const double* __restrict__ part, int nblk, int B, double* __restrict__ out) {
  const int b = blockIdx.x * TPB + threadIdx.x;
  if (b >= B) return;
  double se = 0.0, sd = 0.0;
  for (int k = 0; k < nblk; ++k) {
    se += part[(int64_t(b) * nblk + k) * 2];
    sd += part[(int64_t(b) * nblk + k) * 2 + 1];
  }
  out[2 * b] = se;
  out[2 * b + 1] = sd;
}

// g3 = (2/B) (y3 - e) / ||e_b||^2
__global__ void k_g3(const float* __restrict__ y3, const float* __restrict__ eh, const int32_t* __restrict__ idx,
                     const double* __restrict__ sums, int B, int64_t n3, float* __restrict__ g3) {
  const int64_t k = int64_t(blockIdx.x) * TPB + threadIdx.x;
  if (k >= n3) return;
  const int b = blockIdx.y;
  const int64_t sb = idx ? idx[b] : b;
  const double f = 2.0 / (double(B) * sums[2 * b]);
  g3[int64_t(b) * n3 + k] = float((double(y3[int64_t(b) * n3 + k]) - double(eh[sb * n3 + k])) * f);
}

// Adam; 1 - beta and the bias corrections arrive rounded from FP64 (forming
// 1 - 0.999f in FP32 would be off by 1e-5 relative).
__global__ void k_adam(float* __restrict__ w, const float* __restrict__ g, float* __restrict__ m,
                       float* __restrict__ v, int n, float lr, float b1, float omb1, float b2, float omb2, float eps,
                       float bc1, float bc2) {
  const int t = blockIdx.x * TPB + threadIdx.x;
  if (t >= n) return;
  const float gg = g[t];
  const float mm = b1 * m[t] + omb1 * gg;
  const float vv = b2 * v[t] + omb2 * gg * gg;
  m[t] = mm;
  v[t] = vv;
  w[t] -= lr * (mm / bc1) / (sqrtf(vv / bc2) + eps);
}

// sample b of a planar FP32 batch (sample index idx[b] when given) -> FP64 vector
__global__ void k_sample_f64(const float* __restrict__ src, const int32_t* __restrict__ idx, int b, int64_t n3,
                             double* __restrict__ dst) {
  const int64_t k = int64_t(blockIdx.x) * TPB + threadIdx.x;
  if (k >= n3) return;
  const int64_t sb = idx ? idx[b] : b;
  dst[k] = double(src[sb * n3 + k]);
}

// g3_b = coef * q / sums[1] with sums = {||res||^2, ||r||^2}, as FP32
__global__ void k_scaled_f32(const double* __restrict__ q, const double* __restrict__ sums, double coef, int64_t n3,
                             float* __restrict__ dst) {
  const int64_t k = int64_t(blockIdx.x) * TPB + threadIdx.x;
  if (k >= n3) return;
  dst[k] = float(coef * q[k] / sums[1]);
}

// Minimal-residual loss pieces from sums = {a = <Kc, r>, b = ||Kc||^2, n = ||r||^2}:
// gamma = a / b (0 when b = 0) into sums[3], loss 1 - a^2/(b n) into sums[4],
// output-gradient coefficient -(2/B) a/(n b) into sums[5].
__global__ void k_mr_scalars(double* __restrict__ sums, int B) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const double a = sums[0], b = sums[1], n = sums[2];
  const bool ok = b > 0.0 && n > 0.0;
  sums[3] = ok ? a / b : 0.0;
  sums[4] = ok ? 1.0 - a * a / (b * n) : 1.0;
  sums[5] = ok ? -2.0 / double(B) * a / (n * b) : 0.0;
}

// dst = float(sums[5] * q)
__global__ void k_coef_f32(const double* __restrict__ q, const double* __restrict__ sums, int64_t n3,
                           float* __restrict__ dst) {
  const int64_t k = int64_t(blockIdx.x) * TPB + threadIdx.x;
  if (k >= n3) return;
  dst[k] = float(sums[5] * q[k]);
}

// y = x - sums[3] * z
__global__ void k_sub_gamma(double* __restrict__ y, const double* __restrict__ x, const double* __restrict__ z,
                            const double* __restrict__ sums, int64_t n3) {
  const int64_t k = int64_t(blockIdx.x) * TPB + threadIdx.x;
  if (k >= n3) return;
  y[k] = x[k] - sums[3] * z[k];
}

// pair output: rhat = r / ||r||, ehat = e / ||r|| (FP32)
__global__ void k_pair_write(const double* __restrict__ r, const double* __restrict__ e,
                             const double* __restrict__ nrm2, float* __restrict__ rh, float* __restrict__ eh,
                             int64_t n) {
  const int64_t k = int64_t(blockIdx.x) * TPB + threadIdx.x;
  if (k >= n) return;
  const double inv = 1.0 / sqrt(nrm2[0]);
  rh[k] = float(r[k] * inv);
  eh[k] = float(e[k] * inv);
}

// Stage decision from sc = {||r'||^2, <r', Kc>, ||Kc||^2}: gamma (0 on reject)
// and counters {accepted, rejected}. Accept iff <r',Kc>^2 / ||Kc||^2 >= margin ||r'||^2.
__global__ void k_stage_decide(const double* __restrict__ sc, double margin, double* __restrict__ gamma,
                               double* __restrict__ counters) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const double nr2 = sc[0], num = sc[1], den = sc[2];
  bool ok = nr2 > 0.0 && den > 0.0 && isfinite(den) && isfinite(num);
  if (ok) ok = num * num / den >= margin * nr2;
  gamma[0] = ok ? num / den : 0.0;
  counters[ok ? 0 : 1] += 1.0;
}

__global__ void k_axpy_dev(double* __restrict__ y, const double* __restrict__ a, const double* __restrict__ x,
                           int64_t n) {
  const int64_t k = int64_t(blockIdx.x) * TPB + threadIdx.x;
  if (k >= n) return;
  const double g = a[0];
  if (g != 0.0) y[k] += g * x[k];
}

inline unsigned nb(int64_t n) { return unsigned((n + TPB - 1) / TPB); }
inline int ilog2(int N) {
  int l = 0;
  while ((1 << l) < N) ++l;
  return l;
}

}  // namespace

void* net_dev_alloc(Net& n, size_t bytes) {
  void* p = nullptr;
  const size_t sz = (std::max<size_t>(bytes, 16) + 255) & ~size_t(255);
  if (n.has_ua) {
    p = n.ua.alloc(sz, static_cast<void*>(n.stream), n.ua.user);
    if (!p) throw StatusError(CAV_ERR_OUT_OF_MEMORY, "the caller's allocator returned no block of " +
                                                         std::to_string(sz) + " bytes");
  } else if (hipMalloc(&p, sz) != hipSuccess) {
    (void)hipGetLastError();
    throw StatusError(CAV_ERR_OUT_OF_MEMORY, "hipMalloc of " + std::to_string(bytes) + " bytes failed");
  }
  n.allocs.push_back(p);
  return p;
}

// Returns a block to its source (the work using it is already enqueued on
// the net's stream, which a stream-ordered allocator respects).
static void net_release(Net& n, void* p) {
  if (n.has_ua)
    n.ua.free(p, static_cast<void*>(n.stream), n.ua.user);
  else
    (void)hipFree(p);
}

void net_dev_free(Net& n, void* p) {
  if (!p) return;
  auto it = std::find(n.allocs.begin(), n.allocs.end(), p);
  if (it == n.allocs.end()) return;
  n.allocs.erase(it);
  net_release(n, p);
}

void net_alloc(Net& n, int64_t pix) {
  if (pix <= n.cap_pix) return;
  for (void* p : {(void*)n.d_a1, (void*)n.d_a2, (void*)n.d_y3, (void*)n.d_g3, (void*)n.d_g2, (void*)n.d_g1})
    net_dev_free(n, p);
  n.d_a1 = n.d_a2 = nullptr;
  n.d_y3 = n.d_g3 = n.d_g2 = n.d_g1 = nullptr;
  n.cap_pix = 0;
  n.d_a1 = static_cast<uint16_t*>(net_dev_alloc(n, size_t(pix) * 32 * sizeof(uint16_t)));
  n.d_a2 = static_cast<uint16_t*>(net_dev_alloc(n, size_t(pix) * 32 * sizeof(uint16_t)));
  n.cap_pix = pix;
}

static void net_alloc_train(Net& n, int64_t pix) {
  net_alloc(n, pix);
  if (n.d_g1) return;
  n.d_y3 = static_cast<float*>(net_dev_alloc(n, size_t(n.cap_pix) * 3 * sizeof(float)));
  n.d_g3 = static_cast<float*>(net_dev_alloc(n, size_t(n.cap_pix) * 3 * sizeof(float)));
  n.d_g2 = static_cast<float*>(net_dev_alloc(n, size_t(n.cap_pix) * 32 * sizeof(float)));
  n.d_g1 = static_cast<float*>(net_dev_alloc(n, size_t(n.cap_pix) * 32 * sizeof(float)));
}

void net_pack(Net& n, hipStream_t s) {
  k_pack<<<nb(NET_W), TPB, 0, s>>>(n.d_w, n.d_pk, n.d_w2m);
}

static void forward_hidden(Net& n, int lgN, int B, hipStream_t s) {
  const int N = 1 << lgN;
  dim3 g2((N + L2_TW - 1) / L2_TW, (N + L2_TH - 1) / L2_TH, B);
  k_l2<<<g2, TPB, 0, s>>>(n.d_a1, lgN, n.d_w2m, n.d_a2);
}

void net_forward_f32(Net& n, int N, int B, const float* in, const int32_t* idx, float* out, hipStream_t s) {
  const int lgN = ilog2(N);
  const int64_t n2 = int64_t(N) * N;
  net_alloc(n, n2 * B);
  dim3 g(nb(n2), B);
  k_l1<float><<<g, TPB, 0, s>>>(in, idx, nullptr, lgN, n.d_pk + PK_L1F, n.d_a1);
  forward_hidden(n, lgN, B, s);
  k_l3<float><<<g, TPB, 0, s>>>(n.d_a2, lgN, n.d_pk + PK_L3F, nullptr, out);
}

void net_correct_f64(Net& n, int N, const double* r, const double* nrm2, double* c, double* part, hipStream_t s) {
  const int lgN = ilog2(N);
  const int64_t n2 = int64_t(N) * N;
  net_alloc(n, n2);
  dim3 g(nb(n2), 1);
  k_l1<double><<<g, TPB, 0, s>>>(r, nullptr, nrm2, lgN, n.d_pk + PK_L1F, n.d_a1);
  forward_hidden(n, lgN, 1, s);
  k_l3<double><<<g, TPB, 0, s>>>(n.d_a2, lgN, n.d_pk + PK_L3F, nrm2, c);
  launch_pressure_mean_remove(c, N, part, s);
}

static int loss_blocks(int64_t n3) { return int(std::min<int64_t>(std::max<int64_t>(n3 / 4096, 1), 64)); }

static void ensure_ls(Net& n, int B, int lblk) {
  if (int64_t(B) * (2 * lblk + 2) > n.ls_cap) {
    net_dev_free(n, n.d_ls);
    n.ls_cap = int64_t(B) * (2 * lblk + 2);
    n.d_ls = static_cast<double*>(net_dev_alloc(n, size_t(n.ls_cap) * sizeof(double)));
  }
}

void net_forward_train(Net& n, int N, int B, const float* rhat, const int32_t* idx, hipStream_t s) {
  const int lgN = ilog2(N);
  const int64_t n2 = int64_t(N) * N;
  net_alloc_train(n, n2 * B);
  dim3 g(nb(n2), B);
  k_l1<float><<<g, TPB, 0, s>>>(rhat, idx, nullptr, lgN, n.d_pk + PK_L1F, n.d_a1);
  forward_hidden(n, lgN, B, s);
  k_l3<float><<<g, TPB, 0, s>>>(n.d_a2, lgN, n.d_pk + PK_L3F, nullptr, n.d_y3);
}

double* net_loss_sums(Net& n, int B) {
  ensure_ls(n, B, 1);
  return n.d_ls + int64_t(n.ls_cap) - 2 * B;
}

void net_train_step(Net& n, int N, int B, const float* rhat, const float* ehat, const int32_t* idx, double lr,
                    double* loss, hipStream_t s) {
  const int64_t n2 = int64_t(N) * N, n3 = 3 * n2;
  const int lblk = loss_blocks(n3);
  ensure_ls(n, B, lblk);
  double* lpart = n.d_ls;
  double* lsum = net_loss_sums(n, B);
  net_forward_train(n, N, B, rhat, idx, s);
  // loss and its gradient
  k_loss_partial<<<dim3(lblk, B), TPB, 0, s>>>(n.d_y3, ehat, idx, n3, lpart);
  k_loss_final<<<nb(B), TPB, 0, s>>>(lpart, lblk, B, lsum);
  k_g3<<<dim3(nb(n3), B), TPB, 0, s>>>(n.d_y3, ehat, idx, lsum, B, n3, n.d_g3);
  net_backward_update(n, N, B, rhat, idx, lr, s);
  if (loss) {
    std::vector<double> h(size_t(2) * B);
    CAV_HIP(hipMemcpyAsync(h.data(), lsum, h.size() * sizeof(double), hipMemcpyDeviceToHost, s));
    CAV_HIP(hipStreamSynchronize(s));
    double L = 0.0;
    for (int b = 0; b < B; ++b) L += h[2 * b + 1] / h[2 * b];
    *loss = L / B;
  }
}

// From g3 = dL/dy3 (in n.d_g3): weight gradients, Adam, repack.
void net_backward_update(Net& n, int N, int B, const float* rhat, const int32_t* idx, double lr, hipStream_t s) {
  const int lgN = ilog2(N);
  const int64_t n2 = int64_t(N) * N;
  const int tiles = B * (N / 8) * (N / 8);
  const int nblk = std::min(tiles, 512);
  if (int64_t(nblk) * 9216 > n.wpart_cap) {
    net_dev_free(n, n.d_wpart);
    n.d_wpart = static_cast<float*>(net_dev_alloc(n, size_t(nblk) * 9216 * sizeof(float)));
    n.wpart_cap = int64_t(nblk) * 9216;
  }
  dim3 g(nb(n2), B);
  float* gW1 = n.d_g;
  float* gW2 = n.d_g + 864;
  float* gW3 = n.d_g + 864 + 9216;
  k_wgrad<3><<<nblk, WG<3>::BS, 0, s>>>(n.d_g3, n.d_a2, idx, lgN, B, n.d_wpart);
  k_wgrad_reduce<<<nb(864), TPB, 0, s>>>(n.d_wpart, nblk, 864, gW3);
  k_l3_bwd<<<g, TPB, 0, s>>>(n.d_g3, n.d_a2, lgN, n.d_pk + PK_L3T, n.d_g2);
  k_wgrad<2><<<nblk, WG<2>::BS, 0, s>>>(n.d_g2, n.d_a1, idx, lgN, B, n.d_wpart);
  k_wgrad_reduce<<<nb(9216), TPB, 0, s>>>(n.d_wpart, nblk, 9216, gW2);
  k_l2_bwd<<<g, TPB, 0, s>>>(n.d_g2, n.d_a1, lgN, n.d_pk + PK_L2T, n.d_g1);
  k_wgrad<1><<<nblk, WG<1>::BS, 0, s>>>(n.d_g1, rhat, idx, lgN, B, n.d_wpart);
  k_wgrad_reduce<<<nb(864), TPB, 0, s>>>(n.d_wpart, nblk, 864, gW1);
  // Adam (bias corrections in FP64 on the host)
  const double b1 = 0.9, b2 = 0.999;
  n.adam_t += 1;
  const double bc1 = 1.0 - std::pow(b1, double(n.adam_t)), bc2 = 1.0 - std::pow(b2, double(n.adam_t));
  k_adam<<<nb(NET_W), TPB, 0, s>>>(n.d_w, n.d_g, n.d_m, n.d_v, NET_W, float(lr), float(b1), float(1.0 - b1),
                                   float(b2), float(1.0 - b2), 1e-8f, float(bc1), float(bc2));
  net_pack(n, s);
}

void launch_pair_write(const double* r, const double* e, const double* nrm2, float* rhat, float* ehat, int64_t n,
                       hipStream_t s) {
  k_pair_write<<<nb(n), TPB, 0, s>>>(r, e, nrm2, rhat, ehat, n);
}

void launch_sample_f64(const float* src, const int32_t* idx, int b, int64_t n3, double* dst, hipStream_t s) {
  k_sample_f64<<<nb(n3), TPB, 0, s>>>(src, idx, b, n3, dst);
}

void launch_scaled_f32(const double* q, const double* sums, double coef, int64_t n3, float* dst, hipStream_t s) {
  k_scaled_f32<<<nb(n3), TPB, 0, s>>>(q, sums, coef, n3, dst);
}

void launch_mr_scalars(double* sums, int B, hipStream_t s) { k_mr_scalars<<<1, 64, 0, s>>>(sums, B); }
void launch_coef_f32(const double* q, const double* sums, int64_t n3, float* dst, hipStream_t s) {
  k_coef_f32<<<nb(n3), TPB, 0, s>>>(q, sums, n3, dst);
}
void launch_sub_gamma(double* y, const double* x, const double* z, const double* sums, int64_t n3, hipStream_t s) {
  k_sub_gamma<<<nb(n3), TPB, 0, s>>>(y, x, z, sums, n3);
}

const int32_t* net_upload_index(Net& n, const int32_t* index, int batch, int64_t n_samples, hipStream_t s) {
  if (!index) {
    if (n_samples < batch) throw StatusError(CAV_ERR_INVALID_ARG, "n_samples must cover the batch");
    return nullptr;
  }
  for (int b = 0; b < batch; ++b)
    if (index[b] < 0 || index[b] >= n_samples) throw StatusError(CAV_ERR_INVALID_ARG, "sample index out of range");
  if (n.idx_cap < batch) {
    net_dev_free(n, n.d_idx);
    n.d_idx = static_cast<int32_t*>(net_dev_alloc(n, size_t(batch) * sizeof(int32_t)));
    n.idx_cap = batch;
  }
  CAV_HIP(hipMemcpyAsync(n.d_idx, index, size_t(batch) * sizeof(int32_t), hipMemcpyHostToDevice, s));
  return n.d_idx;
}

void launch_stage_decide(const double* sc, double margin, double* gamma_out, double* counters, hipStream_t s) {
  k_stage_decide<<<1, 64, 0, s>>>(sc, margin, gamma_out, counters);
}

void launch_axpy_dev(double* y, const double* a, const double* x, int64_t n, hipStream_t s) {
  k_axpy_dev<<<nb(n), TPB, 0, s>>>(y, a, x, n);
}

}  // namespace cav

using namespace cav;

#define NET_BEGIN try {
#define NET_END                                                  \
  }                                                              \
  catch (const StatusError& e) {                                 \
    net->n.err = e.msg;                                          \
    return e.st;                                                 \
  }                                                              \
  catch (const HipError& e) {                                    \
    net->n.err = e.msg;                                          \
    return CAV_ERR_HIP;                                          \
  }                                                              \
  catch (const std::bad_alloc&) {                                \
    net->n.err = "host allocation failed";                       \
    return CAV_ERR_OUT_OF_MEMORY;                                \
  }

namespace {
void net_require(bool ok, const char* msg) {
  if (!ok) throw StatusError(CAV_ERR_INVALID_ARG, msg);
}
void check_grid(int N) {
  net_require(N >= 8 && (N & (N - 1)) == 0 && N <= 32768, "N must be a power of two in [8, 32768]");
}
}  // namespace

extern "C" {

cav_status cav_net_create(cav_net* out, int device, void* stream, const cav_allocator* allocator) {
  if (!out) return CAV_ERR_INVALID_ARG;
  if (allocator && (!allocator->alloc || !allocator->free)) return CAV_ERR_INVALID_ARG;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return CAV_ERR_INVALID_ARG;
  if (hipSetDevice(device) != hipSuccess) return CAV_ERR_HIP;
  cav_net net = new (std::nothrow) cav_net_s();
  if (!net) return CAV_ERR_OUT_OF_MEMORY;
  net->n.device = device;
  net->n.stream = static_cast<hipStream_t>(stream);
  if (allocator) {
    net->n.ua = *allocator;
    net->n.has_ua = true;
  }
  Net& n = net->n;
  try {
    n.d_w = static_cast<float*>(net_dev_alloc(n, NET_W * sizeof(float)));
    n.d_g = static_cast<float*>(net_dev_alloc(n, NET_W * sizeof(float)));
    n.d_m = static_cast<float*>(net_dev_alloc(n, NET_W * sizeof(float)));
    n.d_v = static_cast<float*>(net_dev_alloc(n, NET_W * sizeof(float)));
    n.d_pk = static_cast<float*>(net_dev_alloc(n, PK_TOTAL * sizeof(float)));
    n.d_w2m = static_cast<uint16_t*>(net_dev_alloc(n, 9216 * sizeof(uint16_t)));
    CAV_HIP(hipMemsetAsync(n.d_w, 0, NET_W * sizeof(float), n.stream));
    CAV_HIP(hipMemsetAsync(n.d_g, 0, NET_W * sizeof(float), n.stream));
    CAV_HIP(hipMemsetAsync(n.d_m, 0, NET_W * sizeof(float), n.stream));
    CAV_HIP(hipMemsetAsync(n.d_v, 0, NET_W * sizeof(float), n.stream));
    net_pack(n, n.stream);
    CAV_HIP(hipStreamSynchronize(n.stream));
  } catch (...) {
    (void)hipStreamSynchronize(n.stream);
    for (void* p : n.allocs) net_release(n, p);
    delete net;
    return CAV_ERR_OUT_OF_MEMORY;
  }
  *out = net;
  return CAV_OK;
}

cav_status cav_net_destroy(cav_net net) {
  if (!net) return CAV_OK;
  (void)hipSetDevice(net->n.device);
  if (net->n.stream) (void)hipStreamSynchronize(net->n.stream);
  for (void* p : net->n.allocs) net_release(net->n, p);
  delete net;
  return CAV_OK;
}

cav_status cav_net_set_stream(cav_net net, void* stream) {
  if (!net) return CAV_ERR_INVALID_ARG;
  net->n.stream = static_cast<hipStream_t>(stream);
  return CAV_OK;
}

const char* cav_net_last_error(cav_net net) { return net ? net->n.err.c_str() : "null net"; }

cav_status cav_net_set_weights(cav_net net, const float* w) {
  if (!net) return CAV_ERR_INVALID_ARG;
  Net& n = net->n;
  NET_BEGIN
  net_require(w != nullptr, "weights pointer is NULL");
  for (int k = 0; k < NET_W; ++k) net_require(std::isfinite(w[k]), "weights must be finite");
  CAV_HIP(hipMemcpyAsync(n.d_w, w, NET_W * sizeof(float), hipMemcpyHostToDevice, n.stream));
  CAV_HIP(hipMemsetAsync(n.d_m, 0, NET_W * sizeof(float), n.stream));
  CAV_HIP(hipMemsetAsync(n.d_v, 0, NET_W * sizeof(float), n.stream));
  n.adam_t = 0;
  net_pack(n, n.stream);
  CAV_HIP(hipStreamSynchronize(n.stream));
  return CAV_OK;
  NET_END
}

cav_status cav_net_get_weights(cav_net net, float* w, float* grad) {
  if (!net) return CAV_ERR_INVALID_ARG;
  Net& n = net->n;
  NET_BEGIN
  if (w) CAV_HIP(hipMemcpyAsync(w, n.d_w, NET_W * sizeof(float), hipMemcpyDeviceToHost, n.stream));
  if (grad) CAV_HIP(hipMemcpyAsync(grad, n.d_g, NET_W * sizeof(float), hipMemcpyDeviceToHost, n.stream));
  CAV_HIP(hipStreamSynchronize(n.stream));
  return CAV_OK;
  NET_END
}

cav_status cav_net_forward(cav_net net, int32_t N, int32_t batch, const float* in, float* out) {
  if (!net) return CAV_ERR_INVALID_ARG;
  Net& n = net->n;
  NET_BEGIN
  check_grid(N);
  net_require(batch >= 1 && batch <= 65535, "batch must be in [1, 65535]");
  net_require(in && out && in != out, "in and out must be distinct device pointers");
  net_forward_f32(n, N, batch, in, nullptr, out, n.stream);
  CAV_HIP(hipGetLastError());
  return CAV_OK;
  NET_END
}

cav_status cav_net_correct(cav_net net, int32_t N, const double* r, double* c) {
  if (!net) return CAV_ERR_INVALID_ARG;
  Net& n = net->n;
  NET_BEGIN
  check_grid(N);
  net_require(r && c && r != c, "r and c must be distinct device pointers");
  const int64_t len = 3 * int64_t(N) * N;
  const int nbk = dots_blocks(len);
  if (n.red_cap < nbk + 1) {
    net_dev_free(n, n.d_red);
    n.d_red = static_cast<double*>(net_dev_alloc(n, size_t(nbk + 1) * sizeof(double)));
    n.red_cap = nbk + 1;
  }
  launch_dots(r, len, 1, r, len, n.d_red + 1, nbk, n.d_red, n.stream);
  net_correct_f64(n, N, r, n.d_red, c, n.d_red + 1, n.stream);
  CAV_HIP(hipGetLastError());
  return CAV_OK;
  NET_END
}

cav_status cav_net_train_step(cav_net net, int32_t N, int32_t batch, const float* rhat, const float* ehat,
                              const int32_t* index, int64_t n_samples, double lr, double* loss) {
  if (!net) return CAV_ERR_INVALID_ARG;
  Net& n = net->n;
  NET_BEGIN
  check_grid(N);
  net_require(batch >= 1 && batch <= 65535, "batch must be in [1, 65535]");
  net_require(rhat && ehat, "rhat and ehat must be device pointers");
  net_require(std::isfinite(lr) && lr > 0.0, "lr must be positive");
  const int32_t* didx = net_upload_index(n, index, batch, n_samples, n.stream);
  net_train_step(n, N, batch, rhat, ehat, didx, lr, loss, n.stream);
  CAV_HIP(hipGetLastError());
  if (!loss) CAV_HIP(hipStreamSynchronize(n.stream));
  return CAV_OK;
  NET_END
}

}  // extern "C"
