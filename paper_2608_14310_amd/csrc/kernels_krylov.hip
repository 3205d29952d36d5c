// Device-resident FGMRES iteration (Section 5) for graph capture.
//
// One iteration body reads the current column index j from device memory, so
// the same captured launch sequence serves every iteration: copy v_j into a
// fixed input buffer, V-cycle, store z_j, w = K z_j, CGS2 over the first j+1
// columns (the same fixed-order reductions as the host-driven solve), then one
// thread applies the Givens rotations, updates the residual estimate and the
// done flag, and the next basis vector is written only while not done. Once a
// system is done, replays of its body leave its state unchanged.
#include <cmath>

#include "cav_internal.hpp"
#include "dots.hpp"

namespace cav {
namespace {
constexpr int TPB = 256;

__device__ double block_sum_k(double v, double* sh) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) sh[w] = v;
  __syncthreads();
  double r = 0.0;
  if (threadIdx.x == 0)
    for (int i = 0; i < TPB / 64; ++i) r += sh[i];
  __syncthreads();
  return r;
}

__global__ __launch_bounds__(TPB) void k_col_get(const double* __restrict__ V, int64_t ldv,
                                                  const int32_t* __restrict__ gi, double* __restrict__ out,
                                                  int64_t n) {
  const int64_t t = int64_t(blockIdx.x) * TPB + threadIdx.x;
  if (t >= n) return;
  out[t] = V[int64_t(gi[GI_J]) * ldv + t];
}

__global__ __launch_bounds__(TPB) void k_col_put(double* __restrict__ Z, int64_t ldv, const int32_t* __restrict__ gi,
                                                  const double* __restrict__ in, int64_t n) {
  const int64_t t = int64_t(blockIdx.x) * TPB + threadIdx.x;
  if (t >= n) return;
  Z[int64_t(gi[GI_J]) * ldv + t] = in[t];
}

// k = j + 1 dot products of V_i with w: partial sums per block (the same
// chunks and order as the host-driven solve's reduction).
__global__ __launch_bounds__(TPB) void k_dots_partial_dk(const double* __restrict__ V, int64_t ldv,
                                                          const int32_t* __restrict__ gi, const double* __restrict__ w,
                                                          int64_t n, double* __restrict__ part, int nblk) {
  dots_block<TPB>(V, ldv, gi[GI_J] + 1, w, n, part, nblk);
}

__global__ __launch_bounds__(TPB) void k_dots_final_dk(const double* __restrict__ part, int nblk,
                                                        const int32_t* __restrict__ gi, double* __restrict__ out) {
  __shared__ double sh[TPB / 64];
  const int i = blockIdx.x;
  if (i > gi[GI_J]) return;
  double acc = 0.0;
  for (int b = threadIdx.x; b < nblk; b += TPB) acc += part[int64_t(i) * nblk + b];
  const double r = block_sum_k(acc, sh);
  if (threadIdx.x == 0) out[i] = r;
}

__global__ __launch_bounds__(TPB) void k_multi_axpy_dk(double* __restrict__ w, const double* __restrict__ V,
                                                        int64_t ldv, const int32_t* __restrict__ gi,
                                                        const double* __restrict__ coef, int64_t n) {
  const int64_t t = int64_t(blockIdx.x) * TPB + threadIdx.x;
  if (t >= n) return;
  const int k = gi[GI_J] + 1;
  double acc = 0.0;
  for (int i = 0; i < k; ++i) acc += coef[i] * V[int64_t(i) * ldv + t];
  w[t] -= acc;
}

// Givens step of column j (one thread). hd = {h1[0..], h2[0..], ||w||^2}
// at offsets 0, m+2, 2(m+2) with m = max_it.
__global__ void k_givens(int32_t* __restrict__ gi, double* __restrict__ gs, const double* __restrict__ hd,
                         int max_it, double rtol) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  if (gi[GI_DONE]) return;
  const int j = gi[GI_J];
  const int ld = max_it + 1;
  double* H = gs + GS_H(max_it);
  double* cs = gs + GS_CS;
  double* sn = cs + max_it;
  double* g = sn + max_it;
  double* hist = g + (max_it + 1);
  double* col = H + int64_t(j) * ld;
  for (int i = 0; i <= j; ++i) col[i] = hd[i] + hd[(max_it + 2) + i];
  const double hn = sqrt(hd[2 * (max_it + 2)]);
  col[j + 1] = hn;
  for (int i = 0; i < j; ++i) {
    const double a = col[i], b = col[i + 1];
    col[i] = cs[i] * a + sn[i] * b;
    col[i + 1] = -sn[i] * a + cs[i] * b;
  }
  const double rr = hypot(col[j], col[j + 1]);
  const double cj = rr == 0.0 ? 1.0 : col[j] / rr, sj = rr == 0.0 ? 0.0 : col[j + 1] / rr;
  cs[j] = cj;
  sn[j] = sj;
  col[j] = rr;
  col[j + 1] = 0.0;
  g[j + 1] = -sj * g[j];
  g[j] = cj * g[j];
  const double est = fabs(g[j + 1]) / gs[GS_BETA];
  hist[j] = est;
  gs[GS_EST] = est;
  gi[GI_K] = j + 1;
  if (!isfinite(est)) {
    gi[GI_DONE] = 2;
  } else if (est <= rtol || hn == 0.0) {
    gi[GI_CONV] = 1;
    gi[GI_DONE] = 1;
  } else if (j + 1 >= max_it) {
    gi[GI_DONE] = 1;
  } else {
    gs[GS_INVHN] = 1.0 / hn;
    gi[GI_J] = j + 1;
  }
}

// v_{j+1} = w / h_{j+1,j} while not done (j already advanced)
__global__ __launch_bounds__(TPB) void k_next_v(double* __restrict__ V, int64_t ldv, const int32_t* __restrict__ gi,
                                                 const double* __restrict__ w, const double* __restrict__ gs,
                                                 int64_t n) {
  const int64_t t = int64_t(blockIdx.x) * TPB + threadIdx.x;
  if (t >= n || gi[GI_DONE]) return;
  V[int64_t(gi[GI_J]) * ldv + t] = w[t] * gs[GS_INVHN];
}

__global__ void k_gstate_init(int32_t* __restrict__ gi, double* __restrict__ gs, double beta, int max_it) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  for (int i = 0; i < GI_COUNT; ++i) gi[i] = 0;
  gs[GS_BETA] = beta;
  gs[GS_EST] = 1.0;
  gs[GS_INVHN] = 0.0;
  double* g = gs + GS_CS + 2 * max_it;
  g[0] = beta;
}

inline unsigned nb(int64_t n) { return unsigned((n + TPB - 1) / TPB); }
}  // namespace

void launch_gstate_init(int32_t* gi, double* gs, double beta, int max_it, hipStream_t s) {
  k_gstate_init<<<1, 64, 0, s>>>(gi, gs, beta, max_it);
}

// One iteration body up to (not including) the V-cycle, and after it.
void launch_col_get(const double* V, int64_t ldv, const int32_t* gi, double* out, int64_t n, hipStream_t s) {
  k_col_get<<<nb(n), TPB, 0, s>>>(V, ldv, gi, out, n);
}

void launch_arnoldi_dk(const Level& F, double* V, double* Z, int64_t n, const int32_t* gi_c, int32_t* gi, double* gs,
                       const double* zout, double* w, double* part, double* hd, int max_it, double rtol,
                       hipStream_t s) {
  const int nblk = dots_blocks(n);
  k_col_put<<<nb(n), TPB, 0, s>>>(Z, n, gi_c, zout, n);
  launch_apply_op(F, zout, w, nullptr, s);
  double* hd1 = hd;
  double* hd2 = hd + (max_it + 2);
  double* hdn = hd + 2 * (max_it + 2);
  k_dots_partial_dk<<<nblk, TPB, 0, s>>>(V, n, gi_c, w, n, part, nblk);
  k_dots_final_dk<<<max_it + 1, TPB, 0, s>>>(part, nblk, gi_c, hd1);
  k_multi_axpy_dk<<<nb(n), TPB, 0, s>>>(w, V, n, gi_c, hd1, n);
  k_dots_partial_dk<<<nblk, TPB, 0, s>>>(V, n, gi_c, w, n, part, nblk);
  k_dots_final_dk<<<max_it + 1, TPB, 0, s>>>(part, nblk, gi_c, hd2);
  k_multi_axpy_dk<<<nb(n), TPB, 0, s>>>(w, V, n, gi_c, hd2, n);
  launch_dots(w, n, 1, w, n, part, nblk, hdn, s);
  k_givens<<<1, 64, 0, s>>>(gi, gs, hd, max_it, rtol);
  k_next_v<<<nb(n), TPB, 0, s>>>(V, n, gi_c, w, gs, n);
}

}  // namespace cav
