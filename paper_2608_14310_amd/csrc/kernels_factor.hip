// Patch factorisation (Section 3.3) and the coarsest direct solve (Section 4).
//
// Every explicit patch matrix K_p = R_p K_E R_p^T is assembled on the device
// from the level's stencils and E_E rows, equilibrated by one pass of row and
// then column max-norm scaling (powers of two, so exact), and inverted in
// place by Gauss-Jordan elimination with partial pivoting (first maximum on
// ties). The elimination is blocked: NB pivot columns are processed in LDS,
// then the remaining columns receive the accumulated transformation as a
// rank-NB update (one thread per column, coalesced row-major rows, loads in
// batches of rows). Row interchanges are kept as a row map, so rows of the
// work matrix never move; the finalize kernel reads through it.
// kappa_1 = ||K~||_1 ||K~^{-1}||_1 is exact given the inverse. The stored
// operator is M_p = C K~^{-1} R (column-major), which equals K_p^{-1}.
#include <algorithm>
#include <cmath>
#include <utility>

#include "cav_internal.hpp"

namespace cav {

namespace {
constexpr int FT = 256;  // threads per patch workgroup
constexpr int NB = 16;   // Gauss-Jordan panel width
constexpr int NBP = NB + 1;  // LDS row stride of the panel (odd: rows fall in different banks)

__device__ __forceinline__ double pow2_recip(double m) {
  // 2^(1-e) for m = f 2^e, f in [1/2, 1): maps m into [1, 2) exactly
  int e;
  frexp(m, &e);
  return ldexp(1.0, 1 - e);
}

// Entry (a, b) of the rediscretised Stokes part of K_E on an N grid (N >= 4).
__device__ double stencil_entry(int64_t da, int64_t db, const StencilCoef& sc) {
  const int N = sc.N;
  const int64_t n2 = int64_t(N) * N;
  const int ta = int(da / n2), tb = int(db / n2);
  const int64_t ca = da - ta * n2, cb = db - tb * n2;
  const int ia = int(ca / N), ja = int(ca % N), ib = int(cb / N), jb = int(cb % N);
  const int m = N - 1;
  if (ta < 2 && tb < 2) {
    if (ta != tb) return 0.0;
    if (ca == cb) return sc.diag;
    const int di = (ib - ia) & m, dj = (jb - ja) & m;
    if ((dj == 0 && (di == 1 || di == m)) || (di == 0 && (dj == 1 || dj == m))) return -sc.off;
    return 0.0;
  }
  if (ta < 2 && tb == 2) {  // G: (p_ij - p_{i-1,j})/h at u_ij, (p_ij - p_{i,j-1})/h at v_ij
    if (cb == ca) return sc.invh;
    if (ta == 0 && jb == ja && ib == ((ia - 1) & m)) return -sc.invh;
    if (ta == 1 && ib == ia && jb == ((ja - 1) & m)) return -sc.invh;
    return 0.0;
  }
  if (ta == 2 && tb < 2) {  // -D: -(u_{i+1,j} - u_ij + v_{i,j+1} - v_ij)/h
    if (cb == ca) return sc.invh;
    if (tb == 0 && jb == ja && ib == ((ia + 1) & m)) return -sc.invh;
    if (tb == 1 && ib == ia && jb == ((ja + 1) & m)) return -sc.invh;
    return 0.0;
  }
  return 0.0;
}

// Unknowns of the rediscretised Stokes stencil row of unknown d on an N grid
// (the only columns where stencil_entry can be nonzero): for u_ij the u
// neighbours, itself, p_ij and p_{i-1,j}; for v_ij likewise with p_{i,j-1};
// for p_ij the four faces of its cell.
__device__ __forceinline__ int stencil_cols(int32_t d, int N, int32_t* c) {
  const int32_t n2 = N * N, m = N - 1;
  const int t = d / n2, q = d - t * n2, i = q / N, j = q % N;
  auto C = [N](int a, int b) { return a * N + b; };
  if (t == 0) {
    c[0] = d; c[1] = C((i + 1) & m, j); c[2] = C((i - 1) & m, j); c[3] = C(i, (j + 1) & m); c[4] = C(i, (j - 1) & m);
    c[5] = 2 * n2 + q; c[6] = 2 * n2 + C((i - 1) & m, j);
    return 7;
  }
  if (t == 1) {
    c[0] = d; c[1] = n2 + C((i + 1) & m, j); c[2] = n2 + C((i - 1) & m, j); c[3] = n2 + C(i, (j + 1) & m);
    c[4] = n2 + C(i, (j - 1) & m); c[5] = 2 * n2 + q; c[6] = 2 * n2 + C(i, (j - 1) & m);
    return 7;
  }
  c[0] = q; c[1] = C((i + 1) & m, j); c[2] = n2 + q; c[3] = n2 + C(i, (j + 1) & m);
  return 4;
}

struct FactorJob {
  const PatchRec* recs;  // fac = offset into work (row-major n x n)
  double* work;
  const int32_t* slot_dof;
  double* rs;            // per slot
  double* cs;            // per slot
  int32_t* sigma;        // per slot: pivots during elimination, column order afterwards
  int32_t* rowp;         // per slot: physical row of each logical row (interchanges are logical)
  double* kappa;         // per patch id
  int32_t* status;       // per patch id: 0 ok, 1 zero or non-finite pivot
  StencilCoef sc;
  const int32_t* erow_full;
  const int32_t* ecol;
  const double* eval;    // -dt E_E
  int use_ee;
};

__device__ __forceinline__ void argmax_combine(double& v, int& i, double v2, int i2) {
  if (v2 > v || (v2 == v && i2 < i)) {
    v = v2;
    i = i2;
  }
}

// Block-wide argmax of (value, index) for FT threads; result valid in all threads.
__device__ void block_argmax(double& v, int& i, double* sv, int* si) {
  for (int o = 32; o > 0; o >>= 1) {
    const double v2 = __shfl_down(v, o, 64);
    const int i2 = __shfl_down(i, o, 64);
    argmax_combine(v, i, v2, i2);
  }
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) {
    sv[w] = v;
    si[w] = i;
  }
  __syncthreads();
  v = sv[0];
  i = si[0];
  for (int k = 1; k < int(blockDim.x >> 6); ++k) argmax_combine(v, i, sv[k], si[k]);
  __syncthreads();
}

__device__ double block_max(double v, double* sv) {
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_down(v, o, 64));
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) sv[w] = v;
  __syncthreads();
  double r = sv[0];
  for (int k = 1; k < int(blockDim.x >> 6); ++k) r = fmax(r, sv[k]);
  __syncthreads();
  return r;
}

__global__ __launch_bounds__(FT) void k_factor(FactorJob J) {
  extern __shared__ double P[];  // panel, row-major n x NB (row stride NBP), row map and unknowns (n ints each)
  __shared__ double sv[FT / 64];
  __shared__ int si[FT / 64];
  __shared__ int s_flag;
  const PatchRec rec = J.recs[blockIdx.x];
  const int n = rec.n;
  const int tid = threadIdx.x;
  double* W = J.work + rec.fac;
  const int32_t* dofs = J.slot_dof + rec.slot;
  double* rs = J.rs + rec.slot;
  double* cs = J.cs + rec.slot;
  int32_t* piv = J.sigma + rec.slot;
  int32_t* rp = reinterpret_cast<int32_t*>(P + int64_t(n) * NBP);
  int32_t* dl = rp + n;   // the patch's unknowns (sorted), for the column searches
  for (int a = tid; a < n; a += FT) dl[a] = dofs[a];

  // 1. K_p from the stencils: zero, then each row's (at most 7) stencil
  // entries whose column lies in the patch (dofs are sorted)
  for (int64_t e = tid; e < int64_t(n) * n; e += FT) W[e] = 0.0;
  __syncthreads();   // also publishes dl
  for (int a = tid; a < n; a += FT) {
    const int32_t da = dofs[a];
    int32_t cols[7];
    const int nc = stencil_cols(da, J.sc.N, cols);
#pragma unroll
    for (int q = 0; q < 7; ++q) {
      if (q >= nc) break;
      const int32_t g = cols[q];
      int lo = 0, hi = n;
      while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (dl[mid] < g) lo = mid + 1; else hi = mid;
      }
      if (lo < n && dl[lo] == g) W[int64_t(a) * n + lo] = stencil_entry(da, g, J.sc);
    }
  }
  __syncthreads();
  // 2. plus -dt E_E entries whose column lies in the patch (dofs are sorted)
  if (J.use_ee) {
    const int64_t nv = 2 * int64_t(J.sc.N) * J.sc.N;
    for (int a = tid; a < n; a += FT) {
      const int64_t da = dofs[a];
      if (da >= nv) continue;
      for (int q = J.erow_full[da]; q < J.erow_full[da + 1]; ++q) {
        const int32_t g = J.ecol[q];
        int lo = 0, hi = n;
        while (lo < hi) {
          const int mid = (lo + hi) >> 1;
          if (dl[mid] < g) lo = mid + 1; else hi = mid;
        }
        if (lo < n && dl[lo] == g) W[int64_t(a) * n + lo] += J.eval[q];
      }
    }
  }
  __syncthreads();
  // 3. row, then column max-norm equilibration (a wave per row: coalesced;
  // the maximum does not depend on the order)
  {
    const int lane = tid & 63, wv = tid >> 6;
    for (int a = wv; a < n; a += FT / 64) {
      double* Wr = W + int64_t(a) * n;
      double m = 0.0;
      for (int b = lane; b < n; b += 64) m = fmax(m, fabs(Wr[b]));
      for (int o = 32; o > 0; o >>= 1) m = fmax(m, __shfl_xor(m, o, 64));
      const double s = (m > 0.0 && isfinite(m)) ? pow2_recip(m) : 1.0;
      if (lane == 0) rs[a] = s;
      for (int b = lane; b < n; b += 64) Wr[b] *= s;
    }
  }
  __syncthreads();
  double colmax = 0.0;
  constexpr int CB = 8;   // rows whose loads are issued together
  for (int b = tid; b < n; b += FT) {
    double m = 0.0;
    for (int a0 = 0; a0 < n; a0 += CB) {
      double v[CB];
#pragma unroll
      for (int u = 0; u < CB; ++u) v[u] = a0 + u < n ? W[int64_t(a0 + u) * n + b] : 0.0;
#pragma unroll
      for (int u = 0; u < CB; ++u) m = fmax(m, fabs(v[u]));
    }
    const double s = (m > 0.0 && isfinite(m)) ? pow2_recip(m) : 1.0;
    cs[b] = s;
    double sum = 0.0;
    for (int a0 = 0; a0 < n; a0 += CB) {
      double v[CB];
#pragma unroll
      for (int u = 0; u < CB; ++u) v[u] = a0 + u < n ? W[int64_t(a0 + u) * n + b] : 0.0;
#pragma unroll
      for (int u = 0; u < CB; ++u)
        if (a0 + u < n) {
          const double sv = v[u] * s;
          W[int64_t(a0 + u) * n + b] = sv;
          sum += fabs(sv);
        }
    }
    colmax = fmax(colmax, sum);
  }
  const double norm1 = block_max(colmax, sv);
  if (tid == 0) s_flag = 0;
  __syncthreads();

  // 4. blocked in-place Gauss-Jordan with partial pivoting. Row interchanges
  // act on the row map rp (logical row -> physical row of W), so no row of W
  // is ever moved; every arithmetic operation is the one of the physically
  // interchanged elimination.
  for (int a = tid; a < n; a += FT) rp[a] = a;
  __syncthreads();
  for (int c0 = 0; c0 < n; c0 += NB) {
    const int nbp = min(NB, n - c0);
    // columns past nbp stay zero: the rank-NB update below reads all NB of them
    for (int e = tid; e < n * NB; e += FT) {
      const int a = e / NB, t = e % NB;
      P[a * NBP + t] = t < nbp ? W[int64_t(rp[a]) * n + c0 + t] : 0.0;
    }
    __syncthreads();
    for (int t = 0; t < nbp; ++t) {
      const int c = c0 + t;
      double bv = -1.0;
      int bi = n;
      for (int a = c + tid; a < n; a += FT) argmax_combine(bv, bi, fabs(P[a * NBP + t]), a);
      block_argmax(bv, bi, sv, si);
      if (!(bv > 0.0) || !isfinite(bv)) {
        if (tid == 0) s_flag = 1;
        __syncthreads();
        break;
      }
      if (tid == 0) piv[c] = bi;
      if (bi != c && tid < nbp) {
        const double tmp = P[c * NBP + tid];
        P[c * NBP + tid] = P[bi * NBP + tid];
        P[bi * NBP + tid] = tmp;
      }
      if (bi != c && tid == 0) {
        const int32_t tr = rp[c];
        rp[c] = rp[bi];
        rp[bi] = tr;
      }
      __syncthreads();
      const double pv = P[c * NBP + t];
      __syncthreads();
      if (tid < nbp) P[c * NBP + tid] = (tid == t ? 1.0 : P[c * NBP + tid]) / pv;
      __syncthreads();
      for (int a = tid; a < n; a += FT) {
        if (a == c) continue;
        const double f = P[a * NBP + t];
        for (int u = 0; u < nbp; ++u)
          if (u != t) P[a * NBP + u] -= f * P[c * NBP + u];
        P[a * NBP + t] = -f * P[c * NBP + t];
      }
      __syncthreads();
    }
    if (s_flag) break;
    for (int e = tid; e < n * nbp; e += FT) {
      const int a = e / nbp, t = e % nbp;
      W[int64_t(rp[a]) * n + c0 + t] = P[a * NBP + t];
    }
    // rank-nbp update of the other columns: pivot rows <- P11 y, other rows +=
    // P_a y; rows in batches of RC whose loads are issued together
    constexpr int RC = 16;
    for (int j = tid; j < n; j += FT) {
      if (j >= c0 && j < c0 + nbp) continue;
      double y[NB];
#pragma unroll
      for (int t = 0; t < NB; ++t) y[t] = (t < nbp) ? W[int64_t(rp[c0 + t]) * n + j] : 0.0;
      for (int a0 = 0; a0 < n; a0 += RC) {
        double w[RC];
#pragma unroll
        for (int u = 0; u < RC; ++u) w[u] = (a0 + u < n) ? W[int64_t(rp[a0 + u]) * n + j] : 0.0;
#pragma unroll
        for (int u = 0; u < RC; ++u) {
          const int a = a0 + u;
          if (a < n) {
            double s = 0.0;
#pragma unroll
            for (int t = 0; t < NB; ++t) s += P[a * NBP + t] * y[t];
            W[int64_t(rp[a]) * n + j] = (a >= c0 && a < c0 + nbp) ? s : w[u] + s;
          }
        }
      }
    }
    __syncthreads();
  }
  if (s_flag) {
    if (tid == 0) {
      J.status[rec.id] = 1;
      J.kappa[rec.id] = INFINITY;
    }
    return;
  }
  // 5. kappa_1 = ||K~||_1 ||K~^{-1}||_1 (column sums of the inverse, in any column order)
  double cm = 0.0;
  for (int b = tid; b < n; b += FT) {
    double sum = 0.0;
    for (int a = 0; a < n; ++a) sum += fabs(W[int64_t(rp[a]) * n + b]);
    cm = fmax(cm, sum);
  }
  for (int a = tid; a < n; a += FT) J.rowp[rec.slot + a] = rp[a];
  const double ninv = block_max(cm, sv);
  if (tid == 0) {
    J.status[rec.id] = isfinite(ninv) ? 0 : 1;
    J.kappa[rec.id] = norm1 * ninv;
  }
}

// Column order of the inverse: undo the row interchanges on the columns in
// reverse order, sigma = identity then swap(sigma[c], sigma[piv[c]]) for
// c = n-1 .. 0. Done in place over the pivot array: since piv[c] >= c, slot c
// still holds piv[c] when step c runs and slots > c already hold sigma values.
__global__ void k_sigma(const PatchRec* __restrict__ recs, int count, int32_t* __restrict__ sigma,
                        const int32_t* __restrict__ status) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= count) return;
  const PatchRec rec = recs[p];
  if (status[rec.id]) return;
  int32_t* s = sigma + rec.slot;
  for (int c = rec.n - 1; c >= 0; --c) {
    const int q = s[c];
    if (q == c) continue;
    s[c] = s[q];
    s[q] = c;
  }
}

// M[i + j n] = cs[i] * W[rowp[i]][sigma[j]] * rs[j]  (= K_p^{-1}), cast to T.
// 64 x 64 tiles through LDS: W is read along rows (consecutive threads take
// consecutive j) and M written along its columns (consecutive i).
template <typename T>
__global__ __launch_bounds__(256) void k_finalize(const PatchRec* __restrict__ wrec, const PatchRec* __restrict__ orec,
                                                  const double* __restrict__ work, const double* __restrict__ rs,
                                                  const double* __restrict__ cs, const int32_t* __restrict__ sigma,
                                                  const int32_t* __restrict__ rowp, T* __restrict__ out) {
  __shared__ double tile[64][65];
  const PatchRec w = wrec[blockIdx.x];
  const PatchRec o = orec[blockIdx.x];
  const int n = w.n;
  const double* W = work + w.fac;
  const double* r = rs + w.slot;
  const double* c = cs + w.slot;
  const int32_t* sg = sigma + w.slot;
  const int32_t* rw = rowp + w.slot;
  T* M = out + o.fac;
  const int lane = threadIdx.x & 63, grp = threadIdx.x >> 6;
  for (int i0 = 0; i0 < n; i0 += 64)
    for (int j0 = 0; j0 < n; j0 += 64) {
      for (int ii = grp; ii < 64; ii += 4) {
        const int i = i0 + ii, j = j0 + lane;
        if (i < n && j < n) tile[ii][lane] = c[i] * W[int64_t(rw[i]) * n + sg[j]] * r[j];
      }
      __syncthreads();
      for (int jj = grp; jj < 64; jj += 4) {
        const int i = i0 + lane, j = j0 + jj;
        if (i < n && j < n) M[int64_t(j) * n + i] = T(tile[lane][jj]);
      }
      __syncthreads();
    }
}

// The same inverse in the symmetric panel layout (sym_panel_off): only the
// entries on or below the panels' diagonal blocks, i >= 16 floor(j / 16), so
// only the 64 x 64 tiles with j0 <= i0; the writes run down each stored
// column (consecutive i).
template <typename T>
__global__ __launch_bounds__(256) void k_finalize_sym(const PatchRec* __restrict__ wrec,
                                                      const PatchRec* __restrict__ orec,
                                                      const double* __restrict__ work, const double* __restrict__ rs,
                                                      const double* __restrict__ cs, const int32_t* __restrict__ sigma,
                                                      const int32_t* __restrict__ rowp, T* __restrict__ out) {
  __shared__ double tile[64][65];
  const PatchRec w = wrec[blockIdx.x];
  const PatchRec o = orec[blockIdx.x];
  const int n = w.n;
  const double* W = work + w.fac;
  const double* r = rs + w.slot;
  const double* c = cs + w.slot;
  const int32_t* sg = sigma + w.slot;
  const int32_t* rw = rowp + w.slot;
  T* M = out + o.fac;
  const int lane = threadIdx.x & 63, grp = threadIdx.x >> 6;
  for (int i0 = 0; i0 < n; i0 += 64)
    for (int j0 = 0; j0 <= i0; j0 += 64) {
      for (int ii = grp; ii < 64; ii += 4) {
        const int i = i0 + ii, j = j0 + lane;
        if (i < n && j < n && i >= (j & ~(SYM_P - 1))) tile[ii][lane] = c[i] * W[int64_t(rw[i]) * n + sg[j]] * r[j];
      }
      __syncthreads();
      for (int jj = grp; jj < 64; jj += 4) {
        const int i = i0 + lane, j = j0 + jj;
        const int k = j / SYM_P, c0 = SYM_P * k;
        if (i < n && j < n && i >= c0)
          M[sym_panel_off(n, k) + int64_t(j - c0) * (sym_n16(n) - c0) + (i - c0)] = T(tile[lane][jj]);
      }
      __syncthreads();
    }
}

// ------------------------------------------------------ coarsest level ---
// The coarsest level is solved through an explicit inverse (Section 4). K_0 =
// [[A, G], [G^T, 0]] is symmetric with A (velocity) SPD and G^T = -D, and
// its null space is the constant pressure e. Instead of the bordered matrix
// [[K_0, e], [e^T, 0]] we invert the quasi-definite matrix
//   Q = [[A, G], [G^T, -gamma e e^T]],
// whose (2,2) Schur complement -(gamma e e^T + G^T A^{-1} G) is negative
// definite. For any right-hand side the solutions of the two systems share u
// and differ in p by a multiple of e (G e = 0 and e^T G^T = 0), so removing
// the pressure mean from every column of Q^{-1} gives the bordered solution
// operator on (u, p). Every leading principal submatrix of a quasi-definite
// matrix is nonsingular, so Q is inverted by blocked Gauss-Jordan elimination
// that pivots only inside each QB x QB diagonal block: per block, the block
// inverse (one workgroup, LDS), the pivot-row block R = D^{-1} W[C, :] and the
// eliminated column block X, then one rank-QB update of the whole matrix
//   W <- base - X R   (an FP64 tiled product, every entry written once).
constexpr int QB = 64;       // diagonal block of the coarse elimination
constexpr int QT = 64;       // output tile of the coarse update (QT x QT per workgroup)

__global__ void k_coarse_assemble(double* __restrict__ W, int n, StencilCoef sc, double gamma) {
  const int64_t e = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (e >= int64_t(n) * n) return;
  const int a = int(e / n), b = int(e % n);
  const int64_t p0 = 2 * int64_t(sc.N) * sc.N;
  W[e] = stencil_entry(a, b, sc) - ((a >= p0 && b >= p0) ? gamma : 0.0);
}

__global__ void k_coarse_add_ee(double* __restrict__ W, int n, int64_t nv, const int32_t* __restrict__ rptr,
                                const int32_t* __restrict__ col, const double* __restrict__ val) {
  const int64_t a = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (a >= nv) return;
  for (int q = rptr[a]; q < rptr[a + 1]; ++q) W[a * n + col[q]] += val[q];
}

// In-place Gauss-Jordan inverse of the m x m diagonal block W[c0.., c0..]
// (m <= QB) with partial pivoting inside the block (first maximum on ties);
// the column interchanges are undone at the end, so Dv (QB x QB, row-major,
// zero outside m x m) holds the block inverse. status = 1 on a zero or
// non-finite pivot. CQT threads, QB^2 / CQT entries each; the interchange of rows
// k and p is folded into step k's update (row p receives old row k).
constexpr int CQT = 1024;  // threads of the block-inverse workgroup
__global__ __launch_bounds__(CQT) void k_cq_diag(const double* __restrict__ W, int n, int c0, int m,
                                                  double* __restrict__ Dv, int32_t* __restrict__ status) {
  __shared__ double D[QB][QB + 1];
  __shared__ int piv[QB];
  __shared__ double rowk[QB], colk[QB], oldk[QB];
  __shared__ int s_p;
  __shared__ int s_bad;
  const int tid = threadIdx.x;
  for (int e = tid; e < QB * QB; e += CQT) {
    const int i = e / QB, j = e % QB;
    D[i][j] = (i < m && j < m) ? W[int64_t(c0 + i) * n + c0 + j] : 0.0;
  }
  if (tid == 0) s_bad = 0;
  __syncthreads();
  for (int k = 0; k < m; ++k) {
    if (tid < 64) {  // one wavefront finds the pivot row
      double bv = -1.0;
      int bi = m;
      const int i = k + tid;
      if (i < m) {
        bv = fabs(D[i][k]);
        bi = i;
      }
      for (int o = 32; o > 0; o >>= 1) {
        const double v2 = __shfl_down(bv, o, 64);
        const int i2 = __shfl_down(bi, o, 64);
        if (v2 > bv || (v2 == bv && i2 < bi)) {
          bv = v2;
          bi = i2;
        }
      }
      if (tid == 0) {
        s_p = bi;
        piv[k] = bi;
        if (!(bv > 0.0) || !isfinite(bv)) s_bad = 1;
      }
    }
    __syncthreads();
    if (s_bad) break;
    const int p = s_p;
    // pivot row (old row p) scaled; column k after the interchange; old row k
    if (tid < QB) {
      const int j = tid;
      const double pv = D[p][k];
      rowk[j] = (j == k ? 1.0 : D[p][j]) / pv;
      colk[j] = D[j == p ? k : j][k];
      oldk[j] = D[k][j];
    }
    __syncthreads();
    for (int e = tid; e < QB * QB; e += CQT) {
      const int i = e / QB, j = e % QB;
      if (i >= m || j >= m) continue;
      if (i == k) {
        D[i][j] = rowk[j];
      } else {
        const double f = colk[i];
        const double src = (i == p) ? oldk[j] : D[i][j];
        D[i][j] = (j == k) ? -f * rowk[k] : src - f * rowk[j];
      }
    }
    __syncthreads();
  }
  if (s_bad) {
    if (tid == 0) status[0] = 1;
    return;
  }
  // undo the column interchanges: one thread per row applies them in reverse
  if (tid < m)
    for (int k = m - 1; k >= 0; --k) {
      const int p = piv[k];
      if (p != k) {
        const double tmp = D[tid][k];
        D[tid][k] = D[tid][p];
        D[tid][p] = tmp;
      }
    }
  __syncthreads();
  for (int e = tid; e < QB * QB; e += CQT) Dv[e] = D[e / QB][e % QB];
}

// blockIdx.y == 0: R (QB x n, row-major): R[t][j] = (D^{-1} W[C, j])_t for
// j outside C, D^{-1}[t][j - c0] inside; rows t >= m are zero.
// blockIdx.y == 1: X (n x QB, row-major): X[a][t] = W[a][c0 + t] for rows a
// outside C, zero for rows of C and for t >= m.
__global__ __launch_bounds__(256) void k_cq_prep(const double* __restrict__ W, int n, int c0, int m,
                                                 const double* __restrict__ Dv, double* __restrict__ R,
                                                 double* __restrict__ X) {
  const int64_t e = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (e >= int64_t(n) * QB) return;
  if (blockIdx.y == 0) {
    const int t = int(e / n), j = int(e % n);
    double v = 0.0;
    if (t < m) {
      if (j >= c0 && j < c0 + m) {
        v = Dv[t * QB + (j - c0)];
      } else {
        for (int s = 0; s < m; ++s) v += Dv[t * QB + s] * W[int64_t(c0 + s) * n + j];
      }
    }
    R[e] = v;
  } else {
    const int a = int(e / QB), t = int(e % QB);
    X[e] = (t < m && (a < c0 || a >= c0 + m)) ? W[int64_t(a) * n + c0 + t] : 0.0;
  }
}

// W[a][j] <- base(a, j) - sum_t X[a][t] R[t][j] on one QT x QT tile, with
// base = R[a - c0][j] on the rows of C, 0 on the columns of C elsewhere, and
// W[a][j] otherwise. 256 threads; X and R tiles in LDS; the product on FP64
// MFMA 16x16x4: wavefront w takes rows 16w .. 16w + 15 of the tile against
// its four 16-column blocks, 16 k-steps of 4 (operand lanes: A[i][k] in lane
// i + 16 k, B[k][j] in lane j + 16 k; result row k + 4 r, column j of lane
// j + 16 k in its r-th value).
typedef double cq_d4 __attribute__((ext_vector_type(4)));
__global__ __launch_bounds__(256) void k_cq_update(double* __restrict__ W, int n, int c0, int m,
                                                   const double* __restrict__ X, const double* __restrict__ R) {
  __shared__ double Xs[QT][QB + 1];
  __shared__ double Rs[QB][QT + 1];
  const int tid = threadIdx.x;
  const int a0 = blockIdx.y * QT, j0 = blockIdx.x * QT;
  for (int e = tid; e < QT * QB; e += 256) {
    const int r = e / QB, t = e % QB;
    Xs[r][t] = (a0 + r < n) ? X[int64_t(a0 + r) * QB + t] : 0.0;
  }
  for (int e = tid; e < QB * QT; e += 256) {
    const int t = e / QT, cc = e % QT;
    Rs[t][cc] = (j0 + cc < n) ? R[int64_t(t) * n + j0 + cc] : 0.0;
  }
  __syncthreads();
  const int lane = tid & 63, w = tid >> 6, li = lane & 15, lk = lane >> 4;
  cq_d4 acc[4];
#pragma unroll
  for (int ct = 0; ct < 4; ++ct) acc[ct] = cq_d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll 4
  for (int s4 = 0; s4 < QB; s4 += 4) {
    const double av = Xs[16 * w + li][s4 + lk];
#pragma unroll
    for (int ct = 0; ct < 4; ++ct)
      acc[ct] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, Rs[s4 + lk][16 * ct + li], acc[ct], 0, 0, 0);
  }
#pragma unroll
  for (int ct = 0; ct < 4; ++ct)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int a = a0 + 16 * w + lk + 4 * r, j = j0 + 16 * ct + li;
      if (a >= n || j >= n) continue;
      double* wp = W + int64_t(a) * n + j;
      const bool rowC = a >= c0 && a < c0 + m;
      const double base = rowC ? Rs[a - c0][16 * ct + li] : ((j >= c0 && j < c0 + m) ? 0.0 : *wp);
      *wp = base - acc[ct][r];
    }
}

// Remove the pressure mean from every column of the inverse (rows p0..n-1):
// 64 columns per workgroup, four row strides summed in a fixed order.
__global__ __launch_bounds__(256) void k_cq_meanfix(double* __restrict__ W, int n, int p0) {
  __shared__ double part[4][64];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int j = blockIdx.x * 64 + lane;
  double s = 0.0;
  if (j < n)
    for (int a = p0 + w; a < n; a += 4) s += W[int64_t(a) * n + j];
  part[w][lane] = s;
  __syncthreads();
  const double mean = (((part[0][lane] + part[1][lane]) + part[2][lane]) + part[3][lane]) / double(n - p0);
  if (j < n)
    for (int a = p0 + w; a < n; a += 4) W[int64_t(a) * n + j] -= mean;
}

// y[i] = sum_k W[i][k] b[k] for the dense coarsest solution operator
// (row-major n x n). Each wavefront takes CG_ROWS rows; a lane strides the
// columns with four independent loads per row in flight (b comes through the
// cache), then a wavefront reduction adds the lanes.
constexpr int CG_ROWS = 2;
__global__ __launch_bounds__(256) void k_coarse_gemv(const double* __restrict__ W, int n, const double* __restrict__ b,
                                                     double* __restrict__ y) {
  const int lane = threadIdx.x & 63;
  const int row0 = (int(blockIdx.x) * 4 + int(threadIdx.x >> 6)) * CG_ROWS;
  if (row0 >= n) return;  // whole wavefront
  const double* Wr[CG_ROWS];
#pragma unroll
  for (int q = 0; q < CG_ROWS; ++q) Wr[q] = W + int64_t(min(row0 + q, n - 1)) * n;
  double acc[CG_ROWS][4];
#pragma unroll
  for (int q = 0; q < CG_ROWS; ++q)
#pragma unroll
    for (int u = 0; u < 4; ++u) acc[q][u] = 0.0;
  int k = lane;
  for (; k + 192 < n; k += 256) {
    const double bb[4] = {b[k], b[k + 64], b[k + 128], b[k + 192]};
#pragma unroll
    for (int q = 0; q < CG_ROWS; ++q)
#pragma unroll
      for (int u = 0; u < 4; ++u) acc[q][u] += Wr[q][k + 64 * u] * bb[u];
  }
  for (; k < n; k += 64) {
    const double bk = b[k];
#pragma unroll
    for (int q = 0; q < CG_ROWS; ++q) acc[q][0] += Wr[q][k] * bk;
  }
#pragma unroll
  for (int q = 0; q < CG_ROWS; ++q) {
    double t = (acc[q][0] + acc[q][2]) + (acc[q][1] + acc[q][3]);
    for (int o = 32; o > 0; o >>= 1) t += __shfl_down(t, o, 64);
    if (lane == 0 && row0 + q < n) y[row0 + q] = t;
  }
}

inline unsigned nblk(int64_t n, int t = 256) { return unsigned((n + t - 1) / t); }
}  // namespace

// ----------------------------------------------------------------- host ---
namespace {
template <typename T>
T* upload(Ctx& c, const std::vector<T>& h) {
  if (h.empty()) return nullptr;
  T* d = static_cast<T*>(dev_alloc(c, h.size() * sizeof(T)));
  CAV_HIP(hipMemcpyAsync(d, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice, c.stream));
  return d;
}
}  // namespace

// Row table of the 64-row cooperative items: entry item * 64 + q holds the
// unknown of row r0 + q of the item's patch, its E_E entry range (full row
// pointer, velocity rows only) and the row's place in the shared residual
// buffer (slot index; -1 when the patch has a single item), or unknown -1
// past the patch's last row.
__global__ void k_item_rows(const CoopItem* __restrict__ items, int64_t nitems, const int32_t* __restrict__ slot_dof,
                            const int32_t* __restrict__ erow_full, int64_t nv, int4* __restrict__ out) {
  const int64_t t = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (t >= nitems * 64) return;
  const CoopItem it = items[t / 64];
  const int q = int(t % 64);
  int4 v = make_int4(-1, 0, 0, 0);
  if (it.r0 + q < it.rec.n) {
    const int32_t d = slot_dof[it.rec.slot + it.r0 + q];
    const int w = it.rec.n > 64 ? int(it.rec.slot + it.r0 + q) : -1;
    v = d < nv ? make_int4(d, erow_full[d], erow_full[d + 1], w) : make_int4(d, 0, 0, w);
  }
  out[t] = v;
}

FactorPending factor_level_launch(Ctx& c, Level& L, hipStream_t ks) {
  hipStream_t s = c.stream;
  FactorPending fp;
  const int ne = L.n_exp;
  fp.ne = ne;
  // work records: every explicit patch plus the shared standard patch (index ne)
  std::vector<PatchRec> wrec(ne + 1);
  int64_t wtot = 0;
  for (int e = 0; e < ne; ++e) {
    const int n = int(L.exp_off[e + 1] - L.exp_off[e]);
    wrec[e] = PatchRec{n, e, L.exp_off[e], wtot};
    wtot += int64_t(n) * n;
  }
  // shared standard patch of cell (0,0) in role order u_00, u_10, v_00, v_01, p_00
  const int N = L.N;
  const int64_t n2 = int64_t(N) * N;
  std::vector<int32_t> std_dofs = {0, int32_t(N), int32_t(n2), int32_t(n2 + 1), int32_t(2 * n2)};
  fp.std_slot = L.n_slots;
  wrec[ne] = PatchRec{5, ne, fp.std_slot, wtot};
  wtot += 25;
  std::vector<int32_t> slot_all(L.slot_dof_h);
  slot_all.insert(slot_all.end(), std_dofs.begin(), std_dofs.end());
  const int64_t nslot = int64_t(slot_all.size());

  fp.work = static_cast<double*>(dev_alloc(c, size_t(wtot) * sizeof(double)));
  fp.rs = static_cast<double*>(dev_alloc(c, size_t(nslot) * sizeof(double)));
  fp.cs = static_cast<double*>(dev_alloc(c, size_t(nslot) * sizeof(double)));
  fp.sig = static_cast<int32_t*>(dev_alloc(c, size_t(nslot) * sizeof(int32_t)));
  fp.rowp = static_cast<int32_t*>(dev_alloc(c, size_t(nslot) * sizeof(int32_t)));
  fp.kap = static_cast<double*>(dev_alloc(c, size_t(ne + 1) * sizeof(double)));
  fp.sts = static_cast<int32_t*>(dev_alloc(c, size_t(ne + 1) * sizeof(int32_t)));
  fp.slot_all = upload(c, slot_all);
  // largest first, so the long factorisations start first
  std::vector<PatchRec> order(wrec);
  std::stable_sort(order.begin(), order.end(), [](const PatchRec& a, const PatchRec& b) { return a.n > b.n; });
  CAV_HIP(hipMemsetAsync(fp.sts, 0, size_t(ne + 1) * sizeof(int32_t), s));

  FactorJob J{};
  J.work = fp.work;
  J.slot_dof = fp.slot_all;
  J.rs = fp.rs;
  J.cs = fp.cs;
  J.sigma = fp.sig;
  J.rowp = fp.rowp;
  J.kappa = fp.kap;
  J.status = fp.sts;
  J.sc = L.sc;
  J.erow_full = L.d_erow_full;
  J.ecol = L.d_ecol;
  J.eval = L.d_eval;
  // explicit patches with E_E, the shared patch without
  const int nmax = order.empty() ? 5 : order[0].n;
  const size_t lds = size_t(std::max(nmax, 5)) * (NBP * sizeof(double) + 2 * sizeof(int32_t));
  if (lds > 64 * 1024)
    CAV_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(k_factor),
                                hipFuncAttributeMaxDynamicSharedMemorySize, int(lds)));
  for (auto& r : order) (r.id == ne ? fp.std_only : fp.exp_only).push_back(r);
  fp.d_exp = upload(c, fp.exp_only);
  fp.d_std = upload(c, fp.std_only);
  std::vector<PatchRec> all_rec(fp.exp_only);
  all_rec.insert(all_rec.end(), fp.std_only.begin(), fp.std_only.end());
  fp.d_all = upload(c, all_rec);
  if (ks != s) {
    CAV_HIP(hipEventRecord(c.ev_fup, s));
    CAV_HIP(hipStreamWaitEvent(ks, c.ev_fup, 0));
  }
  if (!fp.exp_only.empty()) {
    J.recs = fp.d_exp;
    J.use_ee = 1;
    k_factor<<<unsigned(fp.exp_only.size()), FT, lds, ks>>>(J);
  }
  J.recs = fp.d_std;
  J.use_ee = 0;
  k_factor<<<1, FT, 5 * (NBP * sizeof(double) + 2 * sizeof(int32_t)), ks>>>(J);
  k_sigma<<<nblk(int64_t(all_rec.size()), 64), 64, 0, ks>>>(fp.d_all, int(all_rec.size()), fp.sig, fp.sts);
  CAV_HIP(hipGetLastError());
  return fp;
}

void factor_level_release(Ctx& c, FactorPending& fp) {
  for (void** p : {(void**)&fp.work, (void**)&fp.rs, (void**)&fp.cs, (void**)&fp.sig, (void**)&fp.rowp,
                   (void**)&fp.kap, (void**)&fp.sts, (void**)&fp.slot_all, (void**)&fp.d_exp, (void**)&fp.d_std,
                   (void**)&fp.d_all}) {
    dev_free(c, *p);
    *p = nullptr;
  }
}

void factor_level_finish(Ctx& c, Level& L, FactorPending& fp, int precision, double cond_threshold,
                         cav_factor_stats* st) {
  hipStream_t s = c.stream;
  const int ne = fp.ne;
  const int N = L.N;
  const std::vector<PatchRec>& exp_only = fp.exp_only;
  double* work = fp.work;
  double* rs = fp.rs;
  double* cs = fp.cs;
  int32_t* sig = fp.sig;
  int32_t* rowp = fp.rowp;
  PatchRec* d_std = fp.d_std;
  const int64_t std_slot = fp.std_slot;
  std::vector<double> kap_h(ne + 1);
  std::vector<int32_t> sts_h(ne + 1);
  CAV_HIP(hipMemcpyAsync(kap_h.data(), fp.kap, kap_h.size() * sizeof(double), hipMemcpyDeviceToHost, s));
  CAV_HIP(hipMemcpyAsync(sts_h.data(), fp.sts, sts_h.size() * sizeof(int32_t), hipMemcpyDeviceToHost, s));
  CAV_HIP(hipStreamSynchronize(s));
  for (int e = 0; e <= ne; ++e)
    if (sts_h[e]) {
      throw StatusError(CAV_ERR_SINGULAR_PATCH,
                        "singular patch on level N=" + std::to_string(N) + " (explicit patch " + std::to_string(e) +
                            (e == ne ? ", the shared standard patch)" : ")"));
    }
  // precision per patch, arena offsets, records sorted by size (descending)
  std::vector<PatchRec> w64, o64, w32, o32;
  int64_t a64 = 0, a32 = 0;
  double maxc = 0.0;
  const bool packed = c.layout == CAV_LAYOUT_SYMMETRIC;
  for (auto& r : exp_only) {
    maxc = std::max(maxc, kap_h[r.id]);
    const bool f32 = precision == CAV_PREC_MIXED && kap_h[r.id] <= cond_threshold;
    const int64_t sz = packed ? sym_arena(r.n) : int64_t(r.n) * r.n;
    if (f32) {
      w32.push_back(r);
      o32.push_back(PatchRec{r.n, r.id, r.slot, a32});
      a32 += sz;
    } else {
      w64.push_back(r);
      o64.push_back(PatchRec{r.n, r.id, r.slot, a64});
      a64 += sz;
    }
  }
  if (L.d_f64) dev_free(c, L.d_f64);
  if (L.d_f32) dev_free(c, L.d_f32);
  L.d_f64 = a64 ? static_cast<double*>(dev_alloc(c, size_t(a64) * sizeof(double))) : nullptr;
  L.d_f32 = a32 ? static_cast<float*>(dev_alloc(c, size_t(a32) * sizeof(float))) : nullptr;
  if (!L.d_std_inv) L.d_std_inv = static_cast<double*>(dev_alloc(c, 25 * sizeof(double)));
  if (!w64.empty()) {
    PatchRec* dw = upload(c, w64);
    PatchRec* dout = upload(c, o64);
    if (packed)
      k_finalize_sym<double><<<unsigned(w64.size()), 256, 0, s>>>(dw, dout, work, rs, cs, sig, rowp, L.d_f64);
    else
      k_finalize<double><<<unsigned(w64.size()), 256, 0, s>>>(dw, dout, work, rs, cs, sig, rowp, L.d_f64);
  }
  if (!w32.empty()) {
    PatchRec* dw = upload(c, w32);
    PatchRec* dout = upload(c, o32);
    if (packed)
      k_finalize_sym<float><<<unsigned(w32.size()), 256, 0, s>>>(dw, dout, work, rs, cs, sig, rowp, L.d_f32);
    else
      k_finalize<float><<<unsigned(w32.size()), 256, 0, s>>>(dw, dout, work, rs, cs, sig, rowp, L.d_f32);
  }
  L.packed = packed;
  {
    std::vector<PatchRec> so = {PatchRec{5, ne, std_slot, 0}};
    PatchRec* dout = upload(c, so);
    k_finalize<double><<<1, 256, 0, s>>>(d_std, dout, work, rs, cs, sig, rowp, L.d_std_inv);
  }
  CAV_HIP(hipGetLastError());
  // records the smoother launches, with slots in the level's slot space
  if (L.d_rec64) dev_free(c, L.d_rec64);
  if (L.d_rec32) dev_free(c, L.d_rec32);
  L.rec64_h = o64;
  L.rec32_h = o32;
  // algorithmic bytes of one GEMV launch: the stored factors (n^2 entries, or
  // sym_size(n) in the symmetric layout), slot indices 4n, gathered r 8n, delta 8n
  L.bytes64 = 0;
  L.bytes32 = 0;
  for (auto& r : o64) L.bytes64 += double(packed ? sym_size(r.n) : int64_t(r.n) * r.n) * 8 + 20.0 * r.n;
  for (auto& r : o32) L.bytes32 += double(packed ? sym_size(r.n) : int64_t(r.n) * r.n) * 4 + 20.0 * r.n;
  // multiplicative phases: records in colour order, each naming its arena
  // (not built over symmetric-layout inverses, which those kernels cannot read)
  if (!packed && !L.coloured) colour_explicit(N, L.ee, L);
  if (!packed) {
    std::vector<MultRec> byid(ne);
    for (auto& r : o64) byid[r.id] = MultRec{r.n, 0, r.slot, r.fac};
    for (auto& r : o32) byid[r.id] = MultRec{r.n, 1, r.slot, r.fac};
    std::vector<MultRec> mrec;
    mrec.reserve(L.ph_exp.size());
    L.mrec_max_n = 0;
    for (int32_t e : L.ph_exp) {
      mrec.push_back(byid[e]);
      L.mrec_max_n = std::max(L.mrec_max_n, byid[e].n);
    }
    L.ph_bytes.assign(L.ph_ptr.empty() ? 0 : L.ph_ptr.size() - 1, 0.0);
    L.ph_maxn.assign(L.ph_bytes.size(), 0);
    for (size_t ph = 0; ph + 1 < L.ph_ptr.size(); ++ph)
      for (int32_t q = L.ph_ptr[ph]; q < L.ph_ptr[ph + 1]; ++q) {
        const MultRec& m = mrec[q];
        L.ph_bytes[ph] += double(m.n) * m.n * (m.f32 ? 4 : 8) + 20.0 * m.n;
        L.ph_maxn[ph] = std::max(L.ph_maxn[ph], m.n);
      }
    // LDS of the phase kernel: residual (n doubles) and 16-column block partials
    const int64_t mn = std::max<int32_t>(L.mrec_max_n, 1);
    // residual rows, pre-update values, block partials (doubles), then the unknowns (ints)
    L.mx_lds = size_t(2 * mn + ((mn + 15) / 16) * mn) * sizeof(double) + size_t(mn) * sizeof(int32_t);
    prepare_mult_smoother(L.mx_lds);
    if (L.d_mrec) dev_free(c, L.d_mrec);
    L.d_mrec = upload(c, mrec);
    // split form: one item per (patch, block of 64 rows), grouped by phase
    std::vector<int2> wrk;
    L.ph_wptr.assign(1, 0);
    for (size_t ph = 0; ph + 1 < L.ph_ptr.size(); ++ph) {
      for (int32_t q = L.ph_ptr[ph]; q < L.ph_ptr[ph + 1]; ++q)
        for (int32_t r0 = 0; r0 < mrec[q].n; r0 += 64) wrk.push_back(make_int2(q, r0));
      L.ph_wptr.push_back(int32_t(wrk.size()));
    }
    if (L.d_wrk) dev_free(c, L.d_wrk);
    L.d_wrk = upload(c, wrk);
    // cooperative form: 64- and 128-row blocks, grouped by phase
    const int32_t nrec = int32_t(mrec.size());
    for (int f = 0; f < 2; ++f) {
      const int rb = f == 0 ? 64 : 128;
      std::vector<CoopItem> ci;
      std::vector<int32_t>& wp = f == 0 ? L.ph_wptr : L.ph_wptr2;
      wp.assign(1, 0);
      for (size_t ph = 0; ph + 1 < L.ph_ptr.size(); ++ph) {
        for (int32_t q = L.ph_ptr[ph]; q < L.ph_ptr[ph + 1]; ++q)
          for (int32_t r0 = 0; r0 < mrec[q].n; r0 += rb) ci.push_back(CoopItem{mrec[q], r0, f * nrec + q});
        wp.push_back(int32_t(ci.size()));
      }
      if (L.d_citem[f]) dev_free(c, L.d_citem[f]);
      L.d_citem[f] = upload(c, ci);
      if (f == 0) {
        // the rows of every 64-row item, at item * 64 + row (built on the device)
        if (L.d_irow) dev_free(c, L.d_irow);
        L.d_irow = nullptr;
        if (!ci.empty()) {
          L.d_irow = static_cast<int4*>(dev_alloc(c, ci.size() * 64 * sizeof(int4)));
          k_item_rows<<<nblk(int64_t(ci.size()) * 64, 256), 256, 0, s>>>(L.d_citem[0], int64_t(ci.size()),
                                                                           L.d_slot_dof, L.d_erow_full,
                                                                           2 * int64_t(L.N) * L.N, L.d_irow);
        }
      }
    }
    // two counters per record, one per row-block size: a counter must only
    // ever see rounds of its own k = ceil(n / rows)
    if (L.d_pcnt) dev_free(c, L.d_pcnt);
    const size_t ncnt = 2 * std::max<size_t>(mrec.size(), 1);
    L.d_pcnt = static_cast<unsigned long long*>(dev_alloc(c, ncnt * sizeof(unsigned long long)));
    CAV_HIP(hipMemsetAsync(L.d_pcnt, 0, ncnt * sizeof(unsigned long long), s));
    if (L.d_ph_ptr) dev_free(c, L.d_ph_ptr);
    L.d_ph_ptr = upload(c, L.ph_ptr);
    L.sweep_grid = 0;
    // dataflow sweep: every patch's successors by phase-order index (the
    // patches of later colours that conflict with it) and the number of item
    // completions it waits for per sweep (the 64-row items of all its
    // predecessors); counters start at zero
    {
      const int32_t nr = int32_t(L.ph_exp.size());
      std::vector<int32_t> pos(size_t(ne), -1);
      for (int32_t q = 0; q < nr; ++q) pos[L.ph_exp[q]] = q;
      std::vector<int32_t> need(size_t(std::max(nr, 1)), 0), sptr(size_t(nr) + 1, 0);
      for (int32_t q = 0; q < nr; ++q) {
        const int32_t e = L.ph_exp[q];
        for (int64_t t = L.pred_ptr[e]; t < L.pred_ptr[e + 1]; ++t) {
          const int32_t pq = pos[L.pred[t]];
          need[q] += (mrec[pq].n + 63) / 64;
          ++sptr[pq + 1];
        }
      }
      for (int32_t q = 0; q < nr; ++q) sptr[q + 1] += sptr[q];
      std::vector<int32_t> succ(size_t(std::max(sptr[nr], 1)), 0);
      {
        std::vector<int32_t> fill(sptr.begin(), sptr.end() - 1);
        for (int32_t q = 0; q < nr; ++q) {
          const int32_t e = L.ph_exp[q];
          for (int64_t t = L.pred_ptr[e]; t < L.pred_ptr[e + 1]; ++t) succ[fill[pos[L.pred[t]]]++] = q;
        }
      }
      for (void** pp : {(void**)&L.d_pr_ptr, (void**)&L.d_pr, (void**)&L.d_flow}) {
        if (*pp) dev_free(c, *pp);
        *pp = nullptr;
      }
      // d_pr_ptr: successor offsets (nr + 1), then the completions each patch waits for (nr)
      std::vector<int32_t> tab(sptr);
      tab.insert(tab.end(), need.begin(), need.begin() + nr);
      L.d_pr_ptr = upload(c, tab);
      L.d_pr = upload(c, succ);
      const size_t nf = 1 + std::max<size_t>(mrec.size(), 1);
      L.d_flow = static_cast<unsigned long long*>(dev_alloc(c, nf * sizeof(unsigned long long)));
      launch_zero_u64(L.d_flow, int64_t(nf), s);
      L.flow_base = L.flow_sweep = 0;
      L.flow_items = int64_t(L.ph_wptr.back());
      L.flow_bytes = 0.0;
      for (double v : L.ph_bytes) L.flow_bytes += v;
    }
    if (!c.d_bar) {
      c.d_bar = static_cast<unsigned long long*>(dev_alloc(c, 2 * sizeof(unsigned long long)));
      CAV_HIP(hipMemsetAsync(c.d_bar, 0, 2 * sizeof(unsigned long long), s));
    }
    L.sp_lds = size_t(mn + ((mn + 15) / 16) * 64) * sizeof(double);
    L.cp_lds[0] = size_t(mn + 64 + ((mn + 15) / 16) * 64) * sizeof(double) + 64 * sizeof(int32_t);
    L.cp_lds[1] = size_t(mn + 128 + ((mn + 15) / 16) * 128) * sizeof(double) + 128 * sizeof(int32_t);
    // shared-residual form: room for a 64-row slice of the largest inverse in
    // FP64 (at most 128 KiB, within 159 KiB of LDS); patches whose slice does
    // not fit read the inverse from global memory instead
    {
      const int64_t rest = int64_t(L.cp_lds[0]);
      int64_t pf = std::min<int64_t>(int64_t(64) * mn * 8, 128 * 1024);
      pf = std::min<int64_t>(pf, 159 * 1024 - rest);
      pf = pf >= 64 * 8 * 8 ? (pf / 256) * 256 : 0;
      L.cr_pf = int(pf);
      L.cr_lds = size_t(pf + rest);
    }
    L.mr_lds = size_t(mn) * (16 * sizeof(double) + sizeof(int2) + sizeof(int32_t));
    prepare_mult_smoother(std::max(std::max(L.cp_lds[1], L.cr_lds), L.mr_lds));
  }
  L.d_rec64 = upload(c, o64);
  L.d_rec32 = upload(c, o32);
  // the scratch goes back to the allocator, which reuses a block only after a
  // device-wide synchronisation (the finalize kernels still read it)
  factor_level_release(c, fp);
  if (st) {
    st->n_fp64 += int32_t(w64.size());
    st->n_fp32 += int32_t(w32.size());
    st->max_cond = std::max(st->max_cond, maxc);
    // the entries the smoother reads (the symmetric layout's padding is not)
    for (auto& r : o64) st->factor_bytes += (packed ? sym_size(r.n) : int64_t(r.n) * r.n) * 8;
    for (auto& r : o32) st->factor_bytes += (packed ? sym_size(r.n) : int64_t(r.n) * r.n) * 4;
  }
  L.factored = true;
}

CoarsePending factor_coarse_launch(Ctx& c, hipStream_t s) {
  Level& L = c.lv[0];
  const int N = L.N;
  const int64_t n2 = int64_t(N) * N;
  const int n = int(3 * n2);
  if (n > 4096) throw StatusError(CAV_ERR_INVALID_ARG, "coarsest grid too large for the dense solve (3 N0^2 > 4096)");
  c.nc = n;
  // gamma n0^2 matches the Schur complement scale 4 / (h^2 diag(A_stokes))
  const double gamma = 4.0 * L.sc.invh * L.sc.invh / (L.sc.diag * double(n2));
  CoarsePending cp;
  cp.W = static_cast<double*>(dev_alloc(c, size_t(n) * n * sizeof(double)));
  cp.Dv = static_cast<double*>(dev_alloc(c, size_t(QB) * QB * sizeof(double)));
  cp.R = static_cast<double*>(dev_alloc(c, size_t(QB) * n * sizeof(double)));
  cp.X = static_cast<double*>(dev_alloc(c, size_t(n) * QB * sizeof(double)));
  cp.sts = static_cast<int32_t*>(dev_alloc(c, sizeof(int32_t)));
  double* W = cp.W;
  double* Dv = cp.Dv;
  double* R = cp.R;
  double* X = cp.X;
  int32_t* sts = cp.sts;
  CAV_HIP(hipMemsetAsync(sts, 0, sizeof(int32_t), s));
  k_coarse_assemble<<<nblk(int64_t(n) * n), 256, 0, s>>>(W, n, L.sc, gamma);
  if (L.ee.nnz() > 0) k_coarse_add_ee<<<nblk(2 * n2), 256, 0, s>>>(W, n, 2 * n2, L.d_erow_full, L.d_ecol, L.d_eval);
  const dim3 gu(unsigned((n + QT - 1) / QT), unsigned((n + QT - 1) / QT));
  for (int c0 = 0; c0 < n; c0 += QB) {
    const int m = std::min(QB, n - c0);
    k_cq_diag<<<1, CQT, 0, s>>>(W, n, c0, m, Dv, sts);
    k_cq_prep<<<dim3(nblk(int64_t(n) * QB), 2), 256, 0, s>>>(W, n, c0, m, Dv, R, X);
    k_cq_update<<<gu, 256, 0, s>>>(W, n, c0, m, X, R);
  }
  k_cq_meanfix<<<nblk(n, 64), 256, 0, s>>>(W, n, int(2 * n2));
  CAV_HIP(hipGetLastError());
  return cp;
}

void factor_coarse_release(Ctx& c, CoarsePending& cp) {
  for (void** p : {(void**)&cp.W, (void**)&cp.Dv, (void**)&cp.R, (void**)&cp.X, (void**)&cp.sts}) {
    dev_free(c, *p);
    *p = nullptr;
  }
}

void factor_coarse_finish(Ctx& c, CoarsePending& cp, hipStream_t s) {
  int32_t sts_h = 0;
  CAV_HIP(hipMemcpyAsync(&sts_h, cp.sts, sizeof(int32_t), hipMemcpyDeviceToHost, s));
  CAV_HIP(hipStreamSynchronize(s));
  if (sts_h) {
    factor_coarse_release(c, cp);
    throw StatusError(CAV_ERR_SINGULAR_COARSE, "zero or non-finite pivot in the coarsest factorisation");
  }
  if (c.d_cinv) dev_free(c, c.d_cinv);
  c.d_cinv = cp.W;
  cp.W = nullptr;
  factor_coarse_release(c, cp);
}

void launch_coarse_solve(const Ctx& c, const double* b, double* x, hipStream_t s) {
  const int n = c.nc;
  k_coarse_gemv<<<nblk(n, 4 * CG_ROWS), 256, 0, s>>>(c.d_cinv, n, b, x);
}

}  // namespace cav
