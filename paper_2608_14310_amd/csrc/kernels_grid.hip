// Grid kernels: the reduced operator K_E (stencils plus E_E rows), RT0 /
// bilinear transfers, and fixed-order reductions for the Krylov loop.
// Vectors are [u | v | p], each an N x N block indexed [i][j] with j fastest.
#include "cav_internal.hpp"
#include "dots.hpp"

namespace cav {

namespace {
constexpr int TPB = 256;

__device__ __forceinline__ int wrapi(int a, int N) { return a & (N - 1); }  // N is a power of two

// Stencil rows of K (Eq. intro_saddle) at cell (i, j):
//   (A0 u)_ij = diag u_ij - off (u_{i+-1,j} + u_{i,j+-1}),  (G p)_{u_ij} = (p_ij - p_{i-1,j})/h,
//   (-D u)_ij = -(u_{i+1,j} - u_ij + v_{i,j+1} - v_ij)/h.
// Every thread that writes a u or v row evaluates it with these functions.
__device__ __forceinline__ double stencil_u_row(const StencilCoef& sc, const double* __restrict__ x, int i, int j) {
  const int N = sc.N;
  const int64_t n2 = int64_t(N) * N;
  const double* u = x;
  const double* p = x + 2 * n2;
  const int ip = wrapi(i + 1, N), im = wrapi(i - 1, N), jp = wrapi(j + 1, N), jm = wrapi(j - 1, N);
  const int64_t c = int64_t(i) * N + j;
  return sc.diag * u[c] - sc.off * (u[int64_t(ip) * N + j] + u[int64_t(im) * N + j] + u[int64_t(i) * N + jp] +
                                    u[int64_t(i) * N + jm]) +
         sc.invh * (p[c] - p[int64_t(im) * N + j]);
}

__device__ __forceinline__ double stencil_v_row(const StencilCoef& sc, const double* __restrict__ x, int i, int j) {
  const int N = sc.N;
  const int64_t n2 = int64_t(N) * N;
  const double* v = x + n2;
  const double* p = x + 2 * n2;
  const int ip = wrapi(i + 1, N), im = wrapi(i - 1, N), jp = wrapi(j + 1, N), jm = wrapi(j - 1, N);
  const int64_t c = int64_t(i) * N + j;
  return sc.diag * v[c] - sc.off * (v[int64_t(ip) * N + j] + v[int64_t(im) * N + j] + v[int64_t(i) * N + jp] +
                                    v[int64_t(i) * N + jm]) +
         sc.invh * (p[c] - p[int64_t(i) * N + jm]);
}

// y = K x (b == nullptr) or r = b - K x in one launch. Blocks [0, ncb) take
// one cell per thread and write its p row and each of its u / v rows without
// E_E entries (emask bit 0 / bit 1 clear). The blocks after them take one
// compressed E_E row (of -dt E_E) per EE_LANES lanes, never straddling a
// wavefront: lane l sums the row's entries l, l + EE_LANES, ... in column
// order, an xor tree adds the partial sums (one chain of dependent loads per
// row, a fixed order), and lane 0 writes the whole row, its stencil part plus
// that sum. Every row is written by exactly one thread.
constexpr int EE_LANES = 16;
__global__ __launch_bounds__(TPB) void k_apply_op(StencilCoef sc, int ncb, const uint8_t* __restrict__ emask,
                                                  int nrows, const int32_t* __restrict__ rid,
                                                  const int32_t* __restrict__ rptr, const int32_t* __restrict__ col,
                                                  const double* __restrict__ val, const double* __restrict__ x,
                                                  double* __restrict__ y, const double* __restrict__ b) {
  const int N = sc.N;
  const int64_t n2 = int64_t(N) * N;
  if (int(blockIdx.x) < ncb) {
    const int64_t c = int64_t(blockIdx.x) * TPB + threadIdx.x;
    if (c >= n2) return;
    const int i = int(c / N), j = int(c % N);
    const int ip = wrapi(i + 1, N), jp = wrapi(j + 1, N);
    const double* u = x;
    const double* v = x + n2;
    const uint8_t m = emask ? emask[c] : uint8_t(0);
    const double ap = -sc.invh * ((u[int64_t(ip) * N + j] - u[c]) + (v[int64_t(i) * N + jp] - v[c]));
    if (!(m & 1)) {
      const double au = stencil_u_row(sc, x, i, j);
      y[c] = b ? b[c] - au : au;
    }
    if (!(m & 2)) {
      const double av = stencil_v_row(sc, x, i, j);
      y[n2 + c] = b ? b[n2 + c] - av : av;
    }
    y[2 * n2 + c] = b ? b[2 * n2 + c] - ap : ap;
    return;
  }
  const int64_t g = int64_t(blockIdx.x - ncb) * TPB + threadIdx.x;
  const int64_t t = g / EE_LANES;
  const int l = int(g % EE_LANES);
  double acc = 0.0;
  if (t < nrows)
    for (int q = rptr[t] + l; q < rptr[t + 1]; q += EE_LANES) acc += val[q] * x[col[q]];
#pragma unroll
  for (int o = EE_LANES / 2; o > 0; o >>= 1) acc += __shfl_xor(acc, o, EE_LANES);
  if (t < nrows && l == 0) {
    const int32_t r = rid[t];
    const bool is_v = r >= n2;
    const int64_t c = is_v ? r - n2 : r;
    const int i = int(c / N), j = int(c % N);
    const double st = is_v ? stencil_v_row(sc, x, i, j) : stencil_u_row(sc, x, i, j);
    y[r] = b ? (b[r] - st) - acc : st + acc;
  }
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
  const int ncb = int(nblocks(n2));
  const unsigned grid = unsigned(ncb) + (L.n_erows > 0 ? nblocks(int64_t(L.n_erows) * EE_LANES) : 0u);
  k_apply_op<<<grid, TPB, 0, s>>>(L.sc, ncb, L.n_erows > 0 ? L.d_emask : nullptr, L.n_erows, L.d_erow_id,
                                  L.d_erow_ptr, L.d_ecol, L.d_eval, x, y, b);
}

void launch_stencil(const StencilCoef& sc, const double* x, double* y, const double* b, hipStream_t s) {
  const int ncb = int(nblocks(int64_t(sc.N) * sc.N));
  k_apply_op<<<unsigned(ncb), TPB, 0, s>>>(sc, ncb, nullptr, 0, nullptr, nullptr, nullptr, nullptr, x, y, b);
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
