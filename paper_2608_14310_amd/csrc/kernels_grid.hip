// Grid kernels: the reduced operator K_E (stencils plus E_E rows), RT0 /
// bilinear transfers, and fixed-order reductions for the Krylov loop.
// Vectors are [u | v | p], each an N x N block indexed [i][j] with j fastest.
#include "cav_internal.hpp"
#include "dots.hpp"

namespace cav {

namespace {
constexpr int TPB = 256;

__device__ __forceinline__ int wrapi(int a, int N) { return a & (N - 1); }  // N is a power of two

// y = K x (stencil part) or r = b - K x when b != nullptr. One thread per cell
// computes u_ij, v_ij and p_ij rows (Eq. intro_saddle):
//   (A0 u)_ij = diag u_ij - off (u_{i+-1,j} + u_{i,j+-1}),  (G p)_{u_ij} = (p_ij - p_{i-1,j})/h,
//   (-D u)_ij = -(u_{i+1,j} - u_ij + v_{i,j+1} - v_ij)/h.
__global__ __launch_bounds__(TPB) void k_apply_stencil(StencilCoef sc, const double* __restrict__ x,
                                                       double* __restrict__ y, const double* __restrict__ b) {
  const int N = sc.N;
  const int64_t n2 = int64_t(N) * N;
  const int64_t c = int64_t(blockIdx.x) * TPB + threadIdx.x;
  if (c >= n2) return;
  const int i = int(c / N), j = int(c % N);
  const int ip = wrapi(i + 1, N), im = wrapi(i - 1, N), jp = wrapi(j + 1, N), jm = wrapi(j - 1, N);
  const double* u = x;
  const double* v = x + n2;
  const double* p = x + 2 * n2;
  const double uc = u[c], vc = v[c], pc = p[c];
  const double u_ip = u[int64_t(ip) * N + j], u_im = u[int64_t(im) * N + j];
  const double u_jp = u[int64_t(i) * N + jp], u_jm = u[int64_t(i) * N + jm];
  const double v_ip = v[int64_t(ip) * N + j], v_im = v[int64_t(im) * N + j];
  const double v_jp = v[int64_t(i) * N + jp], v_jm = v[int64_t(i) * N + jm];
  const double p_im = p[int64_t(im) * N + j], p_jm = p[int64_t(i) * N + jm];
  const double au = sc.diag * uc - sc.off * (u_ip + u_im + u_jp + u_jm) + sc.invh * (pc - p_im);
  const double av = sc.diag * vc - sc.off * (v_ip + v_im + v_jp + v_jm) + sc.invh * (pc - p_jm);
  const double ap = -sc.invh * ((u_ip - uc) + (v_jp - vc));
  if (b) {
    y[c] = b[c] - au;
    y[n2 + c] = b[n2 + c] - av;
    y[2 * n2 + c] = b[2 * n2 + c] - ap;
  } else {
    y[c] = au;
    y[n2 + c] = av;
    y[2 * n2 + c] = ap;
  }
}

// Rows of -dt E_E: y[row] += sum val x (apply) or y[row] -= sum val x (residual).
// One thread per compressed row, summing in column order.
__global__ __launch_bounds__(TPB) void k_ee_rows(int nrows, const int32_t* __restrict__ rid,
                                                 const int32_t* __restrict__ rptr, const int32_t* __restrict__ col,
                                                 const double* __restrict__ val, const double* __restrict__ x,
                                                 double* __restrict__ y, double sign) {
  const int t = blockIdx.x * TPB + threadIdx.x;
  if (t >= nrows) return;
  double acc = 0.0;
  for (int q = rptr[t]; q < rptr[t + 1]; ++q) acc += val[q] * x[col[q]];
  y[rid[t]] += sign * acc;
}

// Restriction to the coarse grid (Section 4): velocity R = P^T / 4 of the RT0
// prolongation, pressure = mean of the four child cells.
__global__ __launch_bounds__(TPB) void k_restrict(int Nc, const double* __restrict__ rf, double* __restrict__ bc) {
  const int64_t nc2 = int64_t(Nc) * Nc;
  const int64_t c = int64_t(blockIdx.x) * TPB + threadIdx.x;
  if (c >= nc2) return;
  const int Nf = 2 * Nc;
  const int64_t nf2 = int64_t(Nf) * Nf;
  const int I = int(c / Nc), J = int(c % Nc);
  const int i0 = 2 * I, j0 = 2 * J;
  const int ip = wrapi(i0 + 1, Nf), im = wrapi(i0 - 1, Nf), jp = wrapi(j0 + 1, Nf), jm = wrapi(j0 - 1, Nf);
  const double* u = rf;
  const double* v = rf + nf2;
  const double* p = rf + 2 * nf2;
  auto F = [Nf](int a, int b) { return int64_t(a) * Nf + b; };
  const double ru = u[F(i0, j0)] + u[F(i0, jp)] + 0.5 * (u[F(ip, j0)] + u[F(ip, jp)] + u[F(im, j0)] + u[F(im, jp)]);
  const double rv = v[F(i0, j0)] + v[F(ip, j0)] + 0.5 * (v[F(i0, jp)] + v[F(ip, jp)] + v[F(i0, jm)] + v[F(ip, jm)]);
  const double rp = p[F(i0, j0)] + p[F(i0, jp)] + p[F(ip, j0)] + p[F(ip, jp)];
  bc[c] = 0.25 * ru;
  bc[nc2 + c] = 0.25 * rv;
  bc[2 * nc2 + c] = 0.25 * rp;
}

// xf += P xc: RT0 velocity prolongation and bilinear (9,3,3,1)/16 pressure
// prolongation, periodic.
__global__ __launch_bounds__(TPB) void k_prolong_add(int Nc, const double* __restrict__ xc, double* __restrict__ xf) {
  const int Nf = 2 * Nc;
  const int64_t nf2 = int64_t(Nf) * Nf, nc2 = int64_t(Nc) * Nc;
  const int64_t c = int64_t(blockIdx.x) * TPB + threadIdx.x;
  if (c >= nf2) return;
  const int i = int(c / Nf), j = int(c % Nf);
  const int I = i >> 1, J = j >> 1;
  const int Ip = wrapi(I + 1, Nc), Jp = wrapi(J + 1, Nc);
  auto C = [Nc](int a, int b) { return int64_t(a) * Nc + b; };
  const double* u = xc;
  const double* v = xc + nc2;
  const double* p = xc + 2 * nc2;
  const double pu = (i & 1) ? 0.5 * (u[C(I, J)] + u[C(Ip, J)]) : u[C(I, J)];
  const double pv = (j & 1) ? 0.5 * (v[C(I, J)] + v[C(I, Jp)]) : v[C(I, J)];
  const int sI = wrapi(I + ((i & 1) ? 1 : -1), Nc), sJ = wrapi(J + ((j & 1) ? 1 : -1), Nc);
  const double pp = (9.0 * p[C(I, J)] + 3.0 * p[C(sI, J)] + 3.0 * p[C(I, sJ)] + p[C(sI, sJ)]) * (1.0 / 16.0);
  xf[c] += pu;
  xf[nf2 + c] += pv;
  xf[2 * nf2 + c] += pp;
}

// Block reduction in a fixed tree (deterministic).
__device__ __forceinline__ double block_sum(double v, double* sh) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) sh[wid] = v;
  __syncthreads();
  double r = 0.0;
  if (threadIdx.x == 0) {
    for (int w = 0; w < int(blockDim.x >> 6); ++w) r += sh[w];
  }
  __syncthreads();
  return r;
}

__global__ __launch_bounds__(TPB) void k_dots_partial(const double* __restrict__ V, int64_t ldv, int k,
                                                      const double* __restrict__ w, int64_t n, double* __restrict__ part,
                                                      int nblk) {
  dots_block<TPB>(V, ldv, k, w, n, part, nblk);
}

// out[i] = sum_b part[i * nblk + b], one block per i, fixed order.
__global__ __launch_bounds__(TPB) void k_dots_final(const double* __restrict__ part, int nblk, double* __restrict__ out) {
  __shared__ double sh[TPB / 64];
  const int i = blockIdx.x;
  double acc = 0.0;
  for (int b = threadIdx.x; b < nblk; b += TPB) acc += part[int64_t(i) * nblk + b];
  const double r = block_sum(acc, sh);
  if (threadIdx.x == 0) out[i] = r;
}

// w += sign * sum_i coef[i] V_i
__global__ __launch_bounds__(TPB) void k_multi_axpy(double* __restrict__ w, const double* __restrict__ V, int64_t ldv,
                                                    int k, const double* __restrict__ coef, double sign, int64_t n) {
  const int64_t t = int64_t(blockIdx.x) * TPB + threadIdx.x;
  if (t >= n) return;
  double acc = 0.0;
  for (int i = 0; i < k; ++i) acc += coef[i] * V[int64_t(i) * ldv + t];
  w[t] += sign * acc;
}

__global__ __launch_bounds__(TPB) void k_scale(double* __restrict__ y, const double* __restrict__ x,
                                               const double* __restrict__ denom, int64_t n) {
  const int64_t t = int64_t(blockIdx.x) * TPB + threadIdx.x;
  if (t >= n) return;
  y[t] = x[t] / denom[0];
}

// Pressure mean removal: partial sums, then every block reduces the partials in
// the same order and subtracts the mean from its slice.
__global__ __launch_bounds__(TPB) void k_psum_partial(const double* __restrict__ p, int64_t n2, double* __restrict__ part,
                                                      int nblk) {
  __shared__ double sh[TPB / 64];
  const int64_t chunk = (n2 + nblk - 1) / nblk;
  const int64_t s = int64_t(blockIdx.x) * chunk, e = min(n2, s + chunk);
  double acc = 0.0;
  for (int64_t t = s + threadIdx.x; t < e; t += TPB) acc += p[t];
  const double r = block_sum(acc, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = r;
}

__global__ __launch_bounds__(TPB) void k_psub(double* __restrict__ p, int64_t n2, const double* __restrict__ part, int nblk) {
  __shared__ double sh[TPB / 64];
  __shared__ double mean;
  double acc = 0.0;
  for (int b = threadIdx.x; b < nblk; b += TPB) acc += part[b];
  const double r = block_sum(acc, sh);
  if (threadIdx.x == 0) mean = r / double(n2);
  __syncthreads();
  const int64_t t = int64_t(blockIdx.x) * TPB + threadIdx.x;
  if (t < n2) p[t] -= mean;
}

inline unsigned nblocks(int64_t n) { return unsigned((n + TPB - 1) / TPB); }
}  // namespace

int dots_blocks(int64_t n) {
  int64_t b = (n + 2047) / 2048;   // one tile of TPB x DOT_EPT elements per block up to 2M elements
  if (b < 1) b = 1;
  if (b > 1024) b = 1024;
  return int(b);
}

void launch_apply_op(const Level& L, const double* x, double* y, const double* b, hipStream_t s) {
  const int64_t n2 = int64_t(L.N) * L.N;
  k_apply_stencil<<<nblocks(n2), TPB, 0, s>>>(L.sc, x, y, b);
  if (L.n_erows > 0)
    k_ee_rows<<<nblocks(L.n_erows), TPB, 0, s>>>(L.n_erows, L.d_erow_id, L.d_erow_ptr, L.d_ecol, L.d_eval, x, y,
                                                 b ? -1.0 : 1.0);
}

void launch_stencil(const StencilCoef& sc, const double* x, double* y, const double* b, hipStream_t s) {
  k_apply_stencil<<<nblocks(int64_t(sc.N) * sc.N), TPB, 0, s>>>(sc, x, y, b);
}

void launch_restrict(const Level& Lf, const double* rf, double* bc, hipStream_t s) {
  const int Nc = Lf.N / 2;
  k_restrict<<<nblocks(int64_t(Nc) * Nc), TPB, 0, s>>>(Nc, rf, bc);
}

void launch_prolong_add(const Level& Lf, const double* xc, double* xf, hipStream_t s) {
  const int Nc = Lf.N / 2;
  k_prolong_add<<<nblocks(int64_t(Lf.N) * Lf.N), TPB, 0, s>>>(Nc, xc, xf);
}

void launch_dots(const double* V, int64_t ldv, int k, const double* w, int64_t n, double* part, int nblk, double* out,
                 hipStream_t s) {
  k_dots_partial<<<nblk, TPB, 0, s>>>(V, ldv, k, w, n, part, nblk);
  k_dots_final<<<k, TPB, 0, s>>>(part, nblk, out);
}

void launch_multi_axpy(double* w, const double* V, int64_t ldv, int k, const double* coef, double sign, int64_t n,
                       hipStream_t s) {
  k_multi_axpy<<<nblocks(n), TPB, 0, s>>>(w, V, ldv, k, coef, sign, n);
}

void launch_scale(double* y, const double* x, const double* denom, int64_t n, hipStream_t s) {
  k_scale<<<nblocks(n), TPB, 0, s>>>(y, x, denom, n);
}

__global__ __launch_bounds__(TPB) void k_fill(double* __restrict__ x, double v, int64_t n) {
  const int64_t t = int64_t(blockIdx.x) * TPB + threadIdx.x;
  if (t < n) x[t] = v;
}

void launch_fill(double* x, double v, int64_t n, hipStream_t s) { k_fill<<<nblocks(n), TPB, 0, s>>>(x, v, n); }

void launch_block_sum(const double* x, int64_t n, double* part, double* out, hipStream_t s) {
  const int nblk = dots_blocks(n);
  k_psum_partial<<<nblk, TPB, 0, s>>>(x, n, part, nblk);
  k_dots_final<<<1, TPB, 0, s>>>(part, nblk, out);
}

void launch_pressure_mean_remove(double* x, int N, double* part, hipStream_t s) {
  const int64_t n2 = int64_t(N) * N;
  double* p = x + 2 * n2;
  const int nblk = dots_blocks(n2);
  k_psum_partial<<<nblk, TPB, 0, s>>>(p, n2, part, nblk);
  k_psub<<<nblocks(n2), TPB, 0, s>>>(p, n2, part, nblk);
}

}  // namespace cav
