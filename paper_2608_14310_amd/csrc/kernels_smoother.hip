// Weighted additive CAV smoother (Appendix A, Eq. additive_cav_saddle):
//   w <- w + alpha * sum_p R_p^T Theta_p K_p^{-1} R_p r,  Theta_p = diag(1/cnt),
// then mean-pressure removal (Section 3.3).
//
// Work split on the GPU:
//  * patches without E_E entries are the standard Vanka patch and share one
//    5x5 inverse per level; their contribution is evaluated on the fly, per
//    unknown, by a grid kernel (no storage);
//  * explicit patches (own inverse) run a gather -> GEMV -> per-slot delta
//    kernel, bucketed by size, FP64 or FP32 factors;
//  * unknowns inside an explicit patch ("touched") pull their slot deltas in a
//    fixed order and apply 1/cnt. Every sum has a fixed order (no atomics).
#include "cav_internal.hpp"

namespace cav {

namespace {
constexpr int TPB = 256;

__device__ __forceinline__ int wrapi(int a, int N) { return a & (N - 1); }

// Shared-inverse part. Role order of a standard patch of cell (a,b):
// 0 u_ab, 1 u_{a+1,b}, 2 v_ab, 3 v_{a,b+1}, 4 p_ab. Minv is column-major 5x5.
// For untouched unknowns every incident patch is standard, cnt = 2 (velocity)
// or 1 (pressure), and the weighted result is written; for touched unknowns
// the raw sum over standard incident patches is written for k_touched.
__global__ __launch_bounds__(TPB) void k_std_smooth(int N, const uint8_t* __restrict__ flag,
                                                    const double* __restrict__ Minv, const double* __restrict__ r,
                                                    double* __restrict__ z) {
  const int64_t n2 = int64_t(N) * N;
  const int64_t c = int64_t(blockIdx.x) * TPB + threadIdx.x;
  if (c >= n2) return;
  double M[25];
#pragma unroll
  for (int k = 0; k < 25; ++k) M[k] = Minv[k];
  const int i = int(c / N), j = int(c % N);
  const int ip = wrapi(i + 1, N), im = wrapi(i - 1, N), jp = wrapi(j + 1, N), jm = wrapi(j - 1, N);
  const double* ru = r;
  const double* rv = r + n2;
  const double* rp = r + 2 * n2;
  auto C = [N](int a, int b) { return int64_t(a) * N + b; };
  const uint8_t f0 = flag[c], fL = flag[C(im, j)], fB = flag[C(i, jm)];
  // residual of this cell's standard patch
  double q[5] = {ru[c], ru[C(ip, j)], rv[c], rv[C(i, jp)], rp[c]};
  double su = 0.0, sv = 0.0, sp = 0.0;
  if (!(f0 & 1)) {
    double d0 = 0.0, d2 = 0.0, d4 = 0.0;
#pragma unroll
    for (int k = 0; k < 5; ++k) {
      d0 += M[0 + 5 * k] * q[k];
      d2 += M[2 + 5 * k] * q[k];
      d4 += M[4 + 5 * k] * q[k];
    }
    su += d0;
    sv += d2;
    sp += d4;
  }
  if (!(fL & 1)) {  // cell (i-1, j): u_ij is its right face (role 1)
    const double qL[5] = {ru[C(im, j)], ru[c], rv[C(im, j)], rv[C(im, jp)], rp[C(im, j)]};
    double d1 = 0.0;
#pragma unroll
    for (int k = 0; k < 5; ++k) d1 += M[1 + 5 * k] * qL[k];
    su += d1;
  }
  if (!(fB & 1)) {  // cell (i, j-1): v_ij is its top face (role 3)
    const double qB[5] = {ru[C(i, jm)], ru[C(ip, jm)], rv[C(i, jm)], rv[c], rp[C(i, jm)]};
    double d3 = 0.0;
#pragma unroll
    for (int k = 0; k < 5; ++k) d3 += M[3 + 5 * k] * qB[k];
    sv += d3;
  }
  const bool tu = (f0 & 2) || (fL & 2), tv = (f0 & 2) || (fB & 2);
  z[c] = tu ? su : 0.5 * su;
  z[n2 + c] = tv ? sv : 0.5 * sv;
  z[2 * n2 + c] = sp;
}

// delta[slot + i] = sum_j M[i + j n] r[dof_j]; one workgroup per explicit patch.
// M is column-major so a wavefront reads one contiguous column segment per j.
template <typename T, int NT>
__global__ __launch_bounds__(NT) void k_patch_apply(const PatchRec* __restrict__ recs, const T* __restrict__ arena,
                                                    const int32_t* __restrict__ slot_dof, const double* __restrict__ r,
                                                    double* __restrict__ delta) {
  extern __shared__ unsigned char smem_raw[];
  T* xs = reinterpret_cast<T*>(smem_raw);
  const PatchRec rec = recs[blockIdx.x];
  const int n = rec.n;
  const int32_t* dofs = slot_dof + rec.slot;
  for (int i = threadIdx.x; i < n; i += NT) xs[i] = T(r[dofs[i]]);
  __syncthreads();
  const T* M = arena + rec.fac;
  for (int i0 = 0; i0 < n; i0 += NT) {
    const int i = i0 + threadIdx.x;
    if (i < n) {
      T a0 = T(0), a1 = T(0), a2 = T(0), a3 = T(0);
      const T* col = M + i;
      int jj = 0;
      for (; jj + 4 <= n; jj += 4) {
        a0 += col[int64_t(jj) * n] * xs[jj];
        a1 += col[int64_t(jj + 1) * n] * xs[jj + 1];
        a2 += col[int64_t(jj + 2) * n] * xs[jj + 2];
        a3 += col[int64_t(jj + 3) * n] * xs[jj + 3];
      }
      for (; jj < n; ++jj) a0 += col[int64_t(jj) * n] * xs[jj];
      delta[rec.slot + i] = double((a0 + a1) + (a2 + a3));
    }
  }
}

// z[d] = (1/cnt(d)) * (z[d] + sum over d's slots of delta), slots ascending.
__global__ __launch_bounds__(TPB) void k_touched(int nt, const int32_t* __restrict__ tdof, const double* __restrict__ tinv,
                                                 const int32_t* __restrict__ tptr, const int32_t* __restrict__ tslot,
                                                 const double* __restrict__ delta, double* __restrict__ z) {
  const int t = blockIdx.x * TPB + threadIdx.x;
  if (t >= nt) return;
  const int32_t d = tdof[t];
  double s = z[d];
  for (int q = tptr[t]; q < tptr[t + 1]; ++q) s += delta[tslot[q]];
  z[d] = tinv[t] * s;
}

// x = (zero ? 0 : x) + alpha z
__global__ __launch_bounds__(TPB) void k_update(double* __restrict__ x, const double* __restrict__ z, double alpha,
                                                int zero, int64_t n) {
  const int64_t t = int64_t(blockIdx.x) * TPB + threadIdx.x;
  if (t >= n) return;
  x[t] = (zero ? 0.0 : x[t]) + alpha * z[t];
}

inline unsigned nblocks(int64_t n) { return unsigned((n + TPB - 1) / TPB); }

template <typename T>
void launch_bucketed(const std::vector<PatchRec>& recs_h, const PatchRec* recs_d, const T* arena, const Level& L,
                     const double* r, hipStream_t s) {
  // recs are sorted by n descending; consecutive runs share a workgroup size
  const int total = int(recs_h.size());
  int b0 = 0;
  while (b0 < total) {
    const int nmax = recs_h[b0].n;
    int nt = nmax > 256 ? 512 : nmax > 128 ? 256 : nmax > 64 ? 128 : 64;
    const int lower = nt / 2;
    int b1 = b0;
    while (b1 < total && (recs_h[b1].n > lower || nt == 64)) ++b1;
    const size_t lds = size_t(nmax) * sizeof(T);
    const unsigned grid = unsigned(b1 - b0);
    switch (nt) {
      case 512: k_patch_apply<T, 512><<<grid, 512, lds, s>>>(recs_d + b0, arena, L.d_slot_dof, r, L.d_delta); break;
      case 256: k_patch_apply<T, 256><<<grid, 256, lds, s>>>(recs_d + b0, arena, L.d_slot_dof, r, L.d_delta); break;
      case 128: k_patch_apply<T, 128><<<grid, 128, lds, s>>>(recs_d + b0, arena, L.d_slot_dof, r, L.d_delta); break;
      default: k_patch_apply<T, 64><<<grid, 64, lds, s>>>(recs_d + b0, arena, L.d_slot_dof, r, L.d_delta); break;
    }
    b0 = b1;
  }
}
}  // namespace

void launch_smoother(Ctx& c, Level& L, const double* b, double* x, bool zero_guess, hipStream_t s) {
  const int64_t n2 = int64_t(L.N) * L.N, n = 3 * n2;
  const double* r = b;
  if (!zero_guess) {
    launch_apply_op(L, x, L.d_r, b, s);  // r = b - K x
    r = L.d_r;
  }
  k_std_smooth<<<nblocks(n2), TPB, 0, s>>>(L.N, L.d_cellflag, L.d_std_inv, r, L.d_z);
  if (!L.rec64_h.empty()) launch_bucketed<double>(L.rec64_h, L.d_rec64, L.d_f64, L, r, s);
  if (!L.rec32_h.empty()) launch_bucketed<float>(L.rec32_h, L.d_rec32, L.d_f32, L, r, s);
  if (L.n_touched > 0)
    k_touched<<<nblocks(L.n_touched), TPB, 0, s>>>(L.n_touched, L.d_t_dof, L.d_t_inv, L.d_t_ptr, L.d_t_slot, L.d_delta,
                                                   L.d_z);
  k_update<<<nblocks(n), TPB, 0, s>>>(x, L.d_z, c.alpha, zero_guess ? 1 : 0, n);
  launch_pressure_mean_remove(x, L.N, L.d_part, s);
}

}  // namespace cav
