// Weighted additive CAV smoother (Appendix A, Eq. additive_cav_saddle):
//   w <- w + alpha * sum_p R_p^T Theta_p K_p^{-1} R_p r,  Theta_p = diag(1/cnt),
// then mean-pressure removal (Section 3.3).
//
// Work split on the GPU, two launches per sweep:
//  * k_add_smooth: explicit patches (own inverse, FP64 or FP32) gather their
//    residual, apply the stored inverse and write one delta per slot; in the
//    same launch, patches without E_E entries (the standard Vanka patch, one
//    shared 5x5 inverse per level) are evaluated on the fly per cell, and
//    unknowns outside every explicit patch are updated there;
//  * k_touched: unknowns inside an explicit patch pull their slot deltas in a
//    fixed order, apply 1/cnt and are updated. Every sum has a fixed order
//    (no atomics).
#include <algorithm>

#include "cav_internal.hpp"

namespace cav {

namespace {
constexpr int TPB = 256;
constexpr int MX_THREADS = 1024;

__device__ __forceinline__ int wrapi(int a, int N) { return a & (N - 1); }

// One launch per smoothing step does the explicit patches of both precisions
// and the shared-inverse cells (block ranges [0, P64), [P64, P64 + P32) and
// the rest), and the touched unknowns follow in k_touched, which also applies
// the update. AS_THREADS threads per block.
constexpr int AS_THREADS = 512;
constexpr int AS_UNROLL = 4;

// delta[slot + i] = sum_j M[i + j n] r[dof_j] for one explicit patch. M is
// column-major, so a wavefront reads one contiguous column segment per j.
// Rows sit on lanes (nr = n rounded up to 64); when a patch fills less than
// half the block, G = NT / nr column groups split the columns (group g takes
// j = g, g + G, ...) and their partial sums are added in group order, so
// small patches keep the block's loads in flight. Partial sums use
// AS_UNROLL accumulators added pairwise at the end. STREAM: non-temporal
// loads of the inverse, for a level whose factors exceed the last-level
// cache and are read once per sweep.
// (a compile-time choice: a run-time select between the two loads of the
// same address is merged into one plain load)
template <bool STREAM, typename T>
__device__ __forceinline__ T ld_factor(const T* p) {
  if constexpr (STREAM)
    return __builtin_nontemporal_load(p);
  else
    return *p;
}

template <typename T, int NT, bool STREAM>
__device__ __forceinline__ void patch_gemv(const PatchRec& rec, const T* __restrict__ arena,
                                           const int32_t* __restrict__ slot_dof, const double* __restrict__ r,
                                           double* __restrict__ delta, unsigned char* smem) {
  const int n = rec.n;
  T* xs = reinterpret_cast<T*>(smem);
  T* part = xs + ((n + 1) & ~1);
  const int32_t* dofs = slot_dof + rec.slot;
  for (int i = threadIdx.x; i < n; i += NT) xs[i] = T(r[dofs[i]]);
  __syncthreads();
  const T* M = arena + rec.fac;
  const int nr = ((n + 63) / 64) * 64;
  const int G = nr >= NT ? 1 : NT / nr;
  constexpr int U = AS_UNROLL;
  if (G == 1) {
    for (int i0 = 0; i0 < n; i0 += NT) {
      const int i = i0 + threadIdx.x;
      if (i < n) {
        T a[U];
#pragma unroll
        for (int u = 0; u < U; ++u) a[u] = T(0);
        const T* col = M + i;
        int j = 0;
        for (; j + U <= n; j += U)
#pragma unroll
          for (int u = 0; u < U; ++u) a[u] += ld_factor<STREAM>(col + int64_t(j + u) * n) * xs[j + u];
        for (; j < n; ++j) a[0] += col[int64_t(j) * n] * xs[j];
        delta[rec.slot + i] = double((a[0] + a[2]) + (a[1] + a[3]));
      }
    }
    return;
  }
  const int i = threadIdx.x % nr, g = threadIdx.x / nr;
  T a[U];
#pragma unroll
  for (int u = 0; u < U; ++u) a[u] = T(0);
  if (i < n && g < G) {
    const T* col = M + i;
    int j = g;
    for (; j + (U - 1) * G < n; j += U * G)
#pragma unroll
      for (int u = 0; u < U; ++u) a[u] += ld_factor<STREAM>(col + int64_t(j + u * G) * n) * xs[j + u * G];
    for (; j < n; j += G) a[0] += col[int64_t(j) * n] * xs[j];
  }
  if (g < G) part[g * nr + i] = (a[0] + a[2]) + (a[1] + a[3]);
  __syncthreads();
  if (threadIdx.x < n) {
    T sum = part[threadIdx.x];
    for (int q = 1; q < G; ++q) sum += part[q * nr + threadIdx.x];
    delta[rec.slot + threadIdx.x] = double(sum);
  }
}

// Cross-lane moves of 32-bit words, applied to each word of a T.
template <typename T, typename F>
__device__ __forceinline__ T per_word(T v, F f) {
  constexpr int W = sizeof(T) / 4;
  struct Words { uint32_t w[W]; };
  Words a = __builtin_bit_cast(Words, v);
#pragma unroll
  for (int k = 0; k < W; ++k) a.w[k] = f(a.w[k]);
  return __builtin_bit_cast(T, a);
}
// {x, y} -> {x with lanes 32..63 taken from y's lanes 0..31, y with lanes
// 0..31 taken from x's lanes 32..63} (ROWS = 32), or the same between the odd
// 16-lane rows of x and the even rows of y (ROWS = 16): afterwards x + y is,
// in every lane, its own value plus the partner lane's (l ^ ROWS) of the
// value it keeps (x below the split, y above it).
template <int ROWS, typename T>
__device__ __forceinline__ void swap_halves(T& x, T& y) {
  constexpr int W = sizeof(T) / 4;
  struct Words { uint32_t w[W]; };
  Words a = __builtin_bit_cast(Words, x), b = __builtin_bit_cast(Words, y);
#pragma unroll
  for (int k = 0; k < W; ++k) {
    const auto r = ROWS == 32 ? __builtin_amdgcn_permlane32_swap(a.w[k], b.w[k], false, false)
                              : __builtin_amdgcn_permlane16_swap(a.w[k], b.w[k], false, false);
    a.w[k] = r[0];
    b.w[k] = r[1];
  }
  x = __builtin_bit_cast(T, a);
  y = __builtin_bit_cast(T, b);
}
template <int CTRL, typename T>
__device__ __forceinline__ T dpp(T v) {
  return per_word(v, [](uint32_t w) { return uint32_t(__builtin_amdgcn_update_dpp(0, int(w), CTRL, 0xf, 0xf, false)); });
}
constexpr int DPP_XOR1 = 0xB1;   // quad_perm [1, 0, 3, 2]
constexpr int DPP_XOR2 = 0x4E;   // quad_perm [2, 3, 0, 1]
constexpr int DPP_XOR8 = 0x128;  // row_ror:8 within 16-lane rows

// 16 partial sums per lane (t[q] for panel column q) reduced over the 64
// lanes of a wavefront. Lane bits 5, 4, 3 and 0 halve the values in turn (each
// lane keeps one half, adds its partner's copy of that half and hands the
// other half over), bits 1 and 2 then add partners' sums. Lane l ends with
// the sum of column (l & 1) + 2 ((l >> 3) & 1) + 4 ((l >> 4) & 1) + 8 (l >> 5),
// identical in the four lanes that differ in bits 1 and 2; a fixed order.
template <typename T>
__device__ __forceinline__ T wave_colsum16(T (&t)[SYM_P], int lane) {
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    swap_halves<32>(t[q], t[q + 8]);
    t[q] += t[q + 8];
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    swap_halves<16>(t[q], t[q + 4]);
    t[q] += t[q + 4];
  }
  const bool b3 = lane & 8, b0 = lane & 1;
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    const T keep = b3 ? t[q + 2] : t[q], send = b3 ? t[q] : t[q + 2];
    t[q] = keep + dpp<DPP_XOR8>(send);
  }
  T x;
  {
    const T keep = b0 ? t[1] : t[0], send = b0 ? t[0] : t[1];
    x = keep + dpp<DPP_XOR1>(send);
  }
  x += dpp<DPP_XOR2>(x);
  x += per_word(x, [](uint32_t w) { return uint32_t(__builtin_amdgcn_ds_swizzle(int(w), 0x101F)); });  // lane ^ 4
  return x;
}

// delta[slot + i] = sum_j M[i][j] r[dof_j] for one explicit patch whose
// symmetric inverse is stored in the panel layout (sym_panel_off). Work items
// (64-row chunk R, panel k), dealt round-robin to the block's wavefronts:
// lane l takes row i = 64 R + l and loads its w entries of the panel (one
// contiguous column segment per load), adds M[i][j] q_j over the panel's
// columns (the direct part, every row of the panel) and, for rows below the
// panel's diagonal block, forms M[i][j] q_i, whose sum over the chunk's rows
// is M[j][i]'s contribution to row j (the mirrored part, reduced across the
// wavefront). Both partials go to LDS; row i then adds its direct partials
// over panels k <= i / 16 and its mirrored partials over chunks R >=
// (i / 16) / 4, in that fixed order.
template <typename T, int NT, bool STREAM>
__device__ __forceinline__ void patch_gemv_sym(const PatchRec& rec, const T* __restrict__ arena,
                                               const int32_t* __restrict__ slot_dof, const double* __restrict__ r,
                                               double* __restrict__ delta, unsigned char* smem) {
  constexpr int NW = NT / 64;
  const int n = rec.n;
  const int np = (n + SYM_P - 1) / SYM_P, nr = (n + 63) / 64;
  const int items = sym_items(n);
  T* xs = reinterpret_cast<T*>(smem);
  T* dpart = xs + ((n + 1) & ~1);          // items x 64
  T* tpart = dpart + int64_t(items) * 64;  // items x 16
  const int32_t* dofs = slot_dof + rec.slot;
  for (int i = threadIdx.x; i < n; i += NT) xs[i] = T(r[dofs[i]]);
  __syncthreads();
  const T* M = arena + rec.fac;
  // the item loop is uniform over a wavefront: its indices live in scalar
  // registers and each load is a scalar column base plus the lane's row offset
  const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  int R = 0, base = 0, cnt = np < 4 ? np : 4;
  for (int it = wave; it < items; it += NW) {
    while (it >= base + cnt) {
      base += cnt;
      ++R;
      cnt = 4 * R + 4 < np ? 4 * R + 4 : np;
    }
    const int k = it - base;
    const int c0 = SYM_P * k, w = n - c0 < SYM_P ? n - c0 : SYM_P, m = sym_n16(n) - c0;  // m: column stride
    const int i = 64 * R + lane;
    const bool in = i >= c0 && i < n;
    const T* pan = M + sym_panel_off(n, k);
    // lanes outside the panel read its nearest row (a line the others read
    // anyway: row c0 above the panel, row n - 1 past the patch) and drop it
    const uint32_t off = uint32_t((i < c0 ? c0 : (i < n ? i : n - 1)) - c0);
    T v[SYM_P];
    if (w == SYM_P) {
#pragma unroll
      for (int q = 0; q < SYM_P; ++q) v[q] = ld_factor<STREAM>(pan + int64_t(q) * m + off);
    } else {
#pragma unroll
      for (int q = 0; q < SYM_P; ++q) v[q] = q < w ? ld_factor<STREAM>(pan + int64_t(q) * m + off) : T(0);
    }
#pragma unroll
    for (int q = 0; q < SYM_P; ++q) v[q] = in ? v[q] : T(0);
    T a[4] = {T(0), T(0), T(0), T(0)};
#pragma unroll
    for (int q = 0; q < SYM_P; ++q) a[q & 3] += v[q] * (q < w ? xs[c0 + q] : T(0));
    dpart[it * 64 + lane] = (a[0] + a[2]) + (a[1] + a[3]);
    const T qi = (in && i >= c0 + w) ? xs[i] : T(0);
#pragma unroll
    for (int q = 0; q < SYM_P; ++q) v[q] *= qi;
    const T tsum = wave_colsum16(v, lane);
    if ((lane & 6) == 0) tpart[it * 16 + ((lane & 1) | ((lane >> 2) & 14))] = tsum;
  }
  __syncthreads();
  for (int i = threadIdx.x; i < n; i += NT) {
    const int ri = i >> 6, ki = i / SYM_P;
    int pre = 0;  // first item of chunk ri
    for (int q = 0; q < ri; ++q) pre += 4 * q + 4 < np ? 4 * q + 4 : np;
    T sum = T(0);
    for (int k = 0; k <= ki; ++k) sum += dpart[(pre + k) * 64 + (i & 63)];
    int pr = 0;  // first item of chunk q, for q from 0
    for (int q = 0; q < nr; ++q) {
      if (q >= (ki >> 2)) sum += tpart[(pr + ki) * 16 + (i & 15)];
      pr += 4 * q + 4 < np ? 4 * q + 4 : np;
    }
    delta[rec.slot + i] = double(sum);
  }
}

// Shared-inverse part for cell c = (i, j). Role order of a standard patch of
// cell (a,b): 0 u_ab, 1 u_{a+1,b}, 2 v_ab, 3 v_{a,b+1}, 4 p_ab; Minv is
// column-major 5x5. An unknown outside every explicit patch has only standard
// incident patches (cnt = 2 for velocity, 1 for pressure) and is updated here,
// x <- (zero ? 0 : x) + alpha * sum / cnt; for an unknown inside an explicit
// patch the raw sum over its standard incident patches goes to z for
// k_touched. flag bit 0: the cell's patch is explicit; bits 2, 3, 4: the
// cell's u, v, p unknown is on k_touched's list.
__device__ __forceinline__ void add_std_cell(int N, int64_t c, const uint8_t* __restrict__ flag,
                                         const double* __restrict__ Minv, const double* __restrict__ r,
                                         double* __restrict__ z, double* __restrict__ x, double alpha, bool zero) {
  const int64_t n2 = int64_t(N) * N;
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
  const double q[5] = {ru[c], ru[C(ip, j)], rv[c], rv[C(i, jp)], rp[c]};
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
  const bool tu = f0 & 4, tv = f0 & 8, tp = f0 & 16;
  if (tu) z[c] = su;
  else x[c] = (zero ? 0.0 : x[c]) + alpha * (0.5 * su);
  if (tv) z[n2 + c] = sv;
  else x[n2 + c] = (zero ? 0.0 : x[n2 + c]) + alpha * (0.5 * sv);
  if (tp) z[2 * n2 + c] = sp;
  else x[2 * n2 + c] = (zero ? 0.0 : x[2 * n2 + c]) + alpha * sp;
}

template <bool STREAM, bool SYM>
__global__ __launch_bounds__(AS_THREADS) void k_add_smooth(
    int p64, const PatchRec* __restrict__ rec64, const double* __restrict__ f64, int p32,
    const PatchRec* __restrict__ rec32, const float* __restrict__ f32, const int32_t* __restrict__ slot_dof,
    double* __restrict__ delta, int N, const uint8_t* __restrict__ flag, const double* __restrict__ Minv,
    const double* __restrict__ r, double* __restrict__ z, double* __restrict__ x, double alpha, int zero) {
  extern __shared__ unsigned char smem_raw[];
  const int blk = int(blockIdx.x);
  if (blk < p64) {
    if (SYM)
      patch_gemv_sym<double, AS_THREADS, STREAM>(rec64[blk], f64, slot_dof, r, delta, smem_raw);
    else
      patch_gemv<double, AS_THREADS, STREAM>(rec64[blk], f64, slot_dof, r, delta, smem_raw);
  } else if (blk < p64 + p32) {
    if (SYM)
      patch_gemv_sym<float, AS_THREADS, STREAM>(rec32[blk - p64], f32, slot_dof, r, delta, smem_raw);
    else
      patch_gemv<float, AS_THREADS, STREAM>(rec32[blk - p64], f32, slot_dof, r, delta, smem_raw);
  } else {
    const int64_t c = int64_t(blk - p64 - p32) * AS_THREADS + threadIdx.x;
    if (c < int64_t(N) * N) add_std_cell(N, c, flag, Minv, r, z, x, alpha, zero != 0);
  }
}

// x[d] = (zero ? 0 : x[d]) + alpha / cnt(d) * (z[d] + sum over d's slots of
// delta) for every unknown inside an explicit patch. LANES lanes per touched
// unknown (never straddling a wavefront): lane l sums slots l, l + LANES, ...
// in ascending order and an xor tree adds the partial sums, a fixed order.
// LANES follows the level's mean slots per unknown (8 to 64: the finest 512²
// beam level averages 44), so each lane has a chain of one to three
// dependent loads.
template <int LANES>
__global__ __launch_bounds__(TPB) void k_touched(int nt, const int32_t* __restrict__ tdof, const double* __restrict__ tinv,
                                                 const int32_t* __restrict__ tptr, const int32_t* __restrict__ tslot,
                                                 const double* __restrict__ delta, const double* __restrict__ z,
                                                 double* __restrict__ x, double alpha, int zero) {
  const int64_t g = int64_t(blockIdx.x) * TPB + threadIdx.x;
  const int64_t t = g / LANES;
  const int l = int(g % LANES);
  double s = 0.0;
  if (t < nt)
    for (int q = tptr[t] + l; q < tptr[t + 1]; q += LANES) s += delta[tslot[q]];
#pragma unroll
  for (int o = LANES / 2; o > 0; o >>= 1) s += __shfl_xor(s, o, LANES);
  if (t < nt && l == 0) {
    const int32_t d = tdof[t];
    x[d] = (zero ? 0.0 : x[d]) + alpha * (tinv[t] * (z[d] + s));
  }
}

inline unsigned nblocks(int64_t n) { return unsigned((n + TPB - 1) / TPB); }

// Stencil part of (K_E x) for the unknown of kind kind (0 u, 1 v, 2 p) at
// cell (i, j), without branches: the seven stencil values are loaded at once
// (rows of u and v take their own component's five values and p at the cell
// and its upwind neighbour; p rows take u at the cell and (i+1, j) and v at
// the cell and (i, j+1) in the same slots), both formulas are evaluated with
// the expressions of the MAC stencil, and the kind picks one. Rows of several
// kinds in one wave then cost one round of loads, not one per kind.
__device__ __forceinline__ double krow_at(int kind, int i, int j, const double* __restrict__ x, const StencilCoef& sc) {
  const int N = sc.N;
  const int64_t n2 = int64_t(N) * N;
  const int ip = wrapi(i + 1, N), im = wrapi(i - 1, N), jp = wrapi(j + 1, N), jm = wrapi(j - 1, N);
  auto C = [N](int a, int b) { return int64_t(a) * N + b; };
  const int64_t c = C(i, j);
  const double* w = x + (kind == 1 ? n2 : 0);              // u (u and p rows) or v (v rows)
  const double* q = x + (kind == 2 ? n2 : 2 * n2);         // p (u and v rows) or v (p rows)
  const int64_t q1 = kind == 0 ? C(im, j) : kind == 1 ? C(i, jm) : C(i, jp);
  const double a0 = w[c], a1 = w[C(ip, j)], a2 = w[C(im, j)], a3 = w[C(i, jp)], a4 = w[C(i, jm)];
  const double b0 = q[c], b1 = q[q1];
  const double rp = -sc.invh * ((a1 - a0) + (b1 - b0));
  const double ruv = sc.diag * a0 - sc.off * (a1 + a2 + a3 + a4) + sc.invh * (b0 - b1);
  return kind == 2 ? rp : ruv;
}

// (K_E x)_d for one unknown d >= 0 (3 N^2 < 2^31, so 32-bit divisions): MAC
// stencil row plus the -dt E_E row.
__device__ __forceinline__ double krow(int64_t d, const double* __restrict__ x, const StencilCoef& sc,
                                       const int32_t* __restrict__ erow, const int32_t* __restrict__ ecol,
                                       const double* __restrict__ eval) {
  const uint32_t N = uint32_t(sc.N), n2 = N * N, ud = uint32_t(d);
  const int kind = int(ud / n2);
  const uint32_t c = ud - uint32_t(kind) * n2;
  double acc = krow_at(kind, int(c / N), int(c % N), x, sc);
  if (erow && kind < 2)
    for (int k = erow[d]; k < erow[d + 1]; ++k) acc += eval[k] * x[ecol[k]];
  return acc;
}

// One phase of the multiplicative sweep over explicit patches: one 1024-thread
// workgroup per patch. (1) Residual rows r_i = b_i - (K x)_i of all patch
// unknowns, MX_G lanes per row over the row's E_E entries (indices loaded
// before the gathers) and a fixed-tree reduction. (2) delta = K_p^{-1} r as
// (row, 32-column block) items whose loads are all issued before use, with the
// block partials summed in block order from LDS. (3) x[dofs] += alpha delta.
// Patches of one phase share no unknown and no coupling, so nothing races.
constexpr int MX_G = 8;     // lanes per residual row
constexpr int MX_PER = 8;   // E_E entries a lane loads at once
constexpr int MX_CB = 16;   // columns per GEMV item (keeps the tile in registers at 1024 threads)
constexpr int MX_RB = 64;   // rows per workgroup in the split phase kernels

// Residual rows r = b_d - (K x)_d of the patch unknowns dofs[rr], for rows
// rr = r0 + u * step (u < RR, rr < r1), each computed by one group of MX_G
// lanes (gl = lane in group): E_E entries strided over the group in rounds of
// MX_G * MX_PER (64: one round for every row of the beam workloads), indices
// loaded before the gathers, the stencil part added on lane 0, then a
// fixed-tree reduction; lane 0 passes each row to `emit` with the fourth
// field of its row record. The RR rows of a group are interleaved so that
// their dependent loads are in flight together; each row's own sequence of
// operations (and so its value) does not depend on how rows are grouped,
// which keeps every phase kernel bit-identical.
constexpr int MX_R = 2;
template <int RR = MX_R, typename Src, typename Emit>
__device__ __forceinline__ void mx_residual_rows(Src src, int r0, int step, int r1, int gl, StencilCoef sc,
                                                 const int32_t* __restrict__ ecol, const double* __restrict__ eval,
                                                 const double* __restrict__ b, const double* __restrict__ x,
                                                 Emit emit) {
  int64_t d[RR];
  int q0[RR], q1[RR], qw[RR];
  // src(rr) = {unknown (or -1), E_E entry range, tag passed to emit}: one load per row
#pragma unroll
  for (int u = 0; u < RR; ++u) {
    const int rr = r0 + u * step;
    const int4 q = rr < r1 ? src(rr) : make_int4(-1, 0, 0, 0);
    d[u] = q.x;
    q0[u] = q.y;
    q1[u] = q.z;
    qw[u] = q.w;
  }
  // the stencil part, b and the unknown's own value (lane 0) are loaded now,
  // beside the E_E entries; the sum adds them where it always has
  double stv[RR], bv[RR], xd[RR];
#pragma unroll
  for (int u = 0; u < RR; ++u) {
    const bool own = gl == 0 && d[u] >= 0;
    stv[u] = own ? krow(d[u], x, sc, nullptr, nullptr, nullptr) : 0.0;
    bv[u] = own ? b[d[u]] : 0.0;
    xd[u] = own ? x[d[u]] : 0.0;
  }
  int rounds = 0;
#pragma unroll
  for (int u = 0; u < RR; ++u) rounds = max(rounds, (q1[u] - q0[u] + MX_G * MX_PER - 1) / (MX_G * MX_PER));
  double acc[RR];
#pragma unroll
  for (int u = 0; u < RR; ++u) acc[u] = 0.0;
  for (int k0 = 0; k0 < rounds; ++k0) {
    int cidx[RR][MX_PER];
    double cv[RR][MX_PER];
#pragma unroll
    for (int u = 0; u < RR; ++u)
#pragma unroll
      for (int k = 0; k < MX_PER; ++k) {
        const int q = q0[u] + k0 * MX_G * MX_PER + gl + MX_G * k;
        cidx[u][k] = q < q1[u] ? ecol[q] : -1;
        cv[u][k] = q < q1[u] ? eval[q] : 0.0;
      }
    double xv[RR][MX_PER];
#pragma unroll
    for (int u = 0; u < RR; ++u)
#pragma unroll
      for (int k = 0; k < MX_PER; ++k) xv[u][k] = cidx[u][k] >= 0 ? x[cidx[u][k]] : 0.0;
#pragma unroll
    for (int u = 0; u < RR; ++u)
      if (q0[u] + k0 * MX_G * MX_PER < q1[u]) {
#pragma unroll
        for (int k = 0; k < MX_PER; ++k) acc[u] += cv[u][k] * xv[u][k];
      }
  }
#pragma unroll
  for (int u = 0; u < RR; ++u) {
    if (gl == 0 && d[u] >= 0) acc[u] += stv[u];
#pragma unroll
    for (int o = MX_G / 2; o > 0; o >>= 1) acc[u] += __shfl_down(acc[u], o, MX_G);
    if (gl == 0 && d[u] >= 0) emit(r0 + u * step, bv[u] - acc[u], int32_t(d[u]), xd[u], qw[u]);
  }
}

// Row source over a patch's slots: the unknown and its E_E entry range.
struct SlotRows {
  const int32_t* dofs;
  const int2* sq;
  __device__ __forceinline__ int4 operator()(int rr) const {
    const int2 q = sq[rr];
    return make_int4(dofs[rr], q.x, q.y, 0);
  }
};

// GEMV item (row i, column block cb) of the stored inverse (column-major n x n)
// against r: s0 over even and s1 over odd columns of the block, then s0 + s1.
// Items come in pairs whose loads are all issued before either is used (two
// HBM round trips overlap instead of following each other); each item's
// arithmetic is the same whether it is paired or not.
template <typename T>
__device__ __forceinline__ void mx_load_item(const T* __restrict__ arena, int64_t fac, int n, int i, int cb, bool ok,
                                             T (&m)[MX_CB]) {
  const int j0 = cb * MX_CB, w = ok ? min(MX_CB, n - j0) : 0;
  const T* col = arena + fac + int64_t(j0) * n + i;
#pragma unroll
  for (int jj = 0; jj < MX_CB; ++jj) m[jj] = jj < w ? col[int64_t(jj) * n] : T(0);
}

__device__ __forceinline__ double mx_dot_item(const float (&m)[MX_CB], const double* __restrict__ rp, int n, int cb) {
  const int j0 = cb * MX_CB, w = min(MX_CB, n - j0);
  float s0 = 0.f, s1 = 0.f;
#pragma unroll
  for (int jj = 0; jj < MX_CB; jj += 2) {
    s0 += m[jj] * (jj < w ? float(rp[j0 + jj]) : 0.f);
    s1 += m[jj + 1] * (jj + 1 < w ? float(rp[j0 + jj + 1]) : 0.f);
  }
  return double(s0 + s1);
}

__device__ __forceinline__ double mx_dot_item(const double (&m)[MX_CB], const double* __restrict__ rp, int n, int cb) {
  const int j0 = cb * MX_CB, w = min(MX_CB, n - j0);
  double s0 = 0.0, s1 = 0.0;
#pragma unroll
  for (int jj = 0; jj < MX_CB; jj += 2) {
    s0 += m[jj] * (jj < w ? rp[j0 + jj] : 0.0);
    s1 += m[jj + 1] * (jj + 1 < w ? rp[j0 + jj + 1] : 0.0);
  }
  return s0 + s1;
}

// items t and t + stride (t < count) of an item list mapped by `ij` to
// (row, block); results go to `put(t, value)`.
template <typename T, typename IJ, typename Put>
__device__ __forceinline__ void mx_gemv_pairs(const T* __restrict__ arena, int64_t fac, const double* __restrict__ rp,
                                              int n, int count, int stride, IJ ij, Put put) {
  for (int t = threadIdx.x; t < count; t += 2 * stride) {
    const int t2 = t + stride;
    const bool ok2 = t2 < count;
    int i1, c1, i2 = 0, c2 = 0;
    ij(t, i1, c1);
    if (ok2) ij(t2, i2, c2);
    T m1[MX_CB], m2[MX_CB];
    mx_load_item(arena, fac, n, i1, c1, true, m1);
    mx_load_item(arena, fac, n, i2, c2, ok2, m2);
    put(t, mx_dot_item(m1, rp, n, c1));
    if (ok2) put(t2, mx_dot_item(m2, rp, n, c2));
  }
}

// One phase of the multiplicative sweep over explicit patches, one workgroup
// per patch (NT threads). (1) All residual rows of the patch into LDS.
// (2) delta = K_p^{-1} r as (row, 16-column block) items, block partials in
// LDS. (3) x[dofs] += alpha delta, partials summed in block order.
// Patches of one phase share no unknown and no coupling, so nothing races.
template <int NT>
__device__ __forceinline__ void mx_patch(const MultRec& rec, double* smem, const double* __restrict__ a64,
                                         const float* __restrict__ a32, const int32_t* __restrict__ slot_dof,
                                         StencilCoef sc, const int2* __restrict__ slot_q,
                                         const int32_t* __restrict__ ecol, const double* __restrict__ eval,
                                         const double* __restrict__ b, double* __restrict__ x, double alpha,
                                         const uint8_t* __restrict__ smask) {
  const int n = rec.n;
  const int nb = (n + MX_CB - 1) / MX_CB;
  double* rp = smem;             // n residual rows
  double* xo = smem + n;         // n values of the unknowns before the update
  double* pp = smem + 2 * n;     // nb x n block partials
  int32_t* dd = reinterpret_cast<int32_t*>(pp + int64_t(nb) * n);  // n unknowns
  const SlotRows src{slot_dof + rec.slot, slot_q + rec.slot};
  const int grp = threadIdx.x / MX_G, gl = threadIdx.x % MX_G;
  constexpr int NG = NT / MX_G;
  for (int rb = grp; rb < n; rb += NG * MX_R)
    mx_residual_rows(src, rb, NG, n, gl, sc, ecol, eval, b, x, [&](int rr, double r, int32_t d, double xv, int) {
      rp[rr] = r;
      xo[rr] = xv;
      dd[rr] = d;
    });
  __syncthreads();
  {
    auto ij = [n](int t, int& i, int& cb) {
      i = t % n;
      cb = t / n;
    };
    auto put = [pp](int t, double v) { pp[t] = v; };  // item t = cb * n + i
    if (rec.f32)
      mx_gemv_pairs(a32, rec.fac, rp, n, n * nb, NT, ij, put);
    else
      mx_gemv_pairs(a64, rec.fac, rp, n, n * nb, NT, ij, put);
  }
  __syncthreads();
  for (int i = threadIdx.x; i < n; i += NT) {
    double s = 0.0;
    for (int cb = 0; cb < nb; ++cb) s += pp[int64_t(cb) * n + i];
    if (!smask || smask[rec.slot + i]) x[dd[i]] = xo[i] + alpha * s;
  }
}

// One phase of the multiplicative sweep over explicit patches, one workgroup
// per patch (NT threads). (1) All residual rows of the patch into LDS.
// (2) delta = K_p^{-1} r as (row, 16-column block) items, block partials in
// LDS. (3) x[dofs] += alpha delta, partials summed in block order.
// Patches of one phase share no unknown and no coupling, so nothing races.
template <int NT>
__global__ __launch_bounds__(NT) void k_mult_exp(const MultRec* __restrict__ recs, const double* __restrict__ a64,
                                                 const float* __restrict__ a32, const int32_t* __restrict__ slot_dof,
                                                 StencilCoef sc, const int2* __restrict__ slot_q,
                                                 const int32_t* __restrict__ ecol, const double* __restrict__ eval,
                                                 const double* __restrict__ b, double* __restrict__ x, double alpha,
                                                 const uint8_t* __restrict__ smask) {
  extern __shared__ double smem[];
  const MultRec rec = recs[blockIdx.x];
  mx_patch<NT>(rec, smem, a64, a32, slot_dof, sc, slot_q, ecol, eval, b, x, alpha, smask);
}

// Split form of one phase, for patches too large for one workgroup to stream
// quickly: work items (patch, block of MX_RB rows). k_mult_res writes the
// item's residual rows to the patch's slots of `rbuf` (reads x only);
// k_mult_gemv then reads the whole patch residual from `rbuf`, forms its rows
// of delta with the same items and block order as k_mult_exp, and updates x
// at its rows' unknowns only. The results equal k_mult_exp's bit for bit.
__global__ __launch_bounds__(256) void k_mult_res(const int2* __restrict__ items, const MultRec* __restrict__ recs,
                                                  const int32_t* __restrict__ slot_dof, StencilCoef sc,
                                                  const int2* __restrict__ slot_q, const int32_t* __restrict__ ecol,
                                                  const double* __restrict__ eval, const double* __restrict__ b,
                                                  const double* __restrict__ x, double* __restrict__ rbuf) {
  const int2 it = items[blockIdx.x];
  const MultRec rec = recs[it.x];
  const int r0 = it.y, r1 = min(rec.n, it.y + MX_RB);
  const SlotRows src{slot_dof + rec.slot, slot_q + rec.slot};
  const int grp = threadIdx.x / MX_G, gl = threadIdx.x % MX_G;
  constexpr int NG = 256 / MX_G;
  for (int rb = r0 + grp; rb < r1; rb += NG * MX_R)
    mx_residual_rows(src, rb, NG, r1, gl, sc, ecol, eval, b, x,
                     [&](int rr, double r, int32_t, double, int) { rbuf[rec.slot + rr] = r; });
}

__global__ __launch_bounds__(256) void k_mult_gemv(const int2* __restrict__ items, const MultRec* __restrict__ recs,
                                                   const double* __restrict__ a64, const float* __restrict__ a32,
                                                   const int32_t* __restrict__ slot_dof,
                                                   const double* __restrict__ rbuf, double* __restrict__ x,
                                                   double alpha, const uint8_t* __restrict__ smask) {
  extern __shared__ double smem[];
  const int2 it = items[blockIdx.x];
  const MultRec rec = recs[it.x];
  const int n = rec.n;
  const int nb = (n + MX_CB - 1) / MX_CB;
  const int r0 = it.y, nr = min(MX_RB, n - r0);
  double* rp = smem;             // n
  double* pp = smem + n;         // nb x MX_RB block partials
  for (int j = threadIdx.x; j < n; j += 256) rp[j] = rbuf[rec.slot + j];
  __syncthreads();
  {
    auto ij = [nr, r0](int t, int& i, int& cb) {
      i = r0 + t % nr;
      cb = t / nr;
    };
    auto put = [pp, nr](int t, double v) { pp[(t / nr) * MX_RB + t % nr] = v; };
    if (rec.f32)
      mx_gemv_pairs(a32, rec.fac, rp, n, nr * nb, 256, ij, put);
    else
      mx_gemv_pairs(a64, rec.fac, rp, n, nr * nb, 256, ij, put);
  }
  __syncthreads();
  const int32_t* dofs = slot_dof + rec.slot;
  for (int ii = threadIdx.x; ii < nr; ii += 256) {
    double s = 0.0;
    for (int cb = 0; cb < nb; ++cb) s += pp[cb * MX_RB + ii];
    if (!smask || smask[rec.slot + r0 + ii]) x[dofs[r0 + ii]] += alpha * s;
  }
}

// Cooperative form of one phase: a patch with n > RB rows is spread over
// k = ceil(n / RB) workgroups, item (patch, first row r0). Every workgroup of
// the patch forms all n residual rows in LDS (the same rows and arithmetic as
// k_mult_exp), then the k workgroups meet at a barrier on the patch's arrival
// counter, so that no unknown of the patch is written before all of them have
// read x; each then forms its RB rows of delta (items and block order as in
// k_mult_exp) and updates x at those rows. The results equal k_mult_exp's bit
// for bit. The counter only grows: an arrival that reads `old` waits for the
// end of its round, (old / k + 1) k, so it never needs a reset. The k
// workgroups of a patch are consecutive items of one launch, which the
// dispatcher places in order; the wait is bounded all the same, and a timeout
// sets err and leaves x unwritten (the host reports the failure).
template <int RB>
__global__ __launch_bounds__(1024) void k_mult_coop(const CoopItem* __restrict__ items,
                                                    const double* __restrict__ a64, const float* __restrict__ a32,
                                                    const int32_t* __restrict__ slot_dof, StencilCoef sc,
                                                    const int2* __restrict__ slot_q, const int32_t* __restrict__ ecol,
                                                    const double* __restrict__ eval, const double* __restrict__ b,
                                                    double* __restrict__ x, double alpha,
                                                    const uint8_t* __restrict__ smask,
                                                    unsigned long long* __restrict__ cnt, int* __restrict__ err,
                                                    unsigned limit) {
  constexpr int NT = 1024;
  extern __shared__ double smem[];
  __shared__ int s_ok;
  const CoopItem it = items[blockIdx.x];
  const MultRec rec = it.rec;
  const int n = rec.n;
  const int nb = (n + MX_CB - 1) / MX_CB;
  const int k = (n + RB - 1) / RB;
  const int r0 = it.r0, nr = min(RB, n - r0);
  double* rp = smem;             // n residual rows
  double* xo = smem + n;         // RB values of this item's unknowns before the update
  double* pp = xo + RB;          // nb x RB block partials
  int32_t* dd = reinterpret_cast<int32_t*>(pp + nb * RB);  // RB unknowns
  const SlotRows src{slot_dof + rec.slot, slot_q + rec.slot};
  const int grp = threadIdx.x / MX_G, gl = threadIdx.x % MX_G;
  constexpr int NG = NT / MX_G;
  for (int rb = grp; rb < n; rb += NG * MX_R)
    mx_residual_rows(src, rb, NG, n, gl, sc, ecol, eval, b, x, [&](int rr, double r, int32_t d, double xv, int) {
      rp[rr] = r;
      if (rr >= r0 && rr < r0 + nr) {
        xo[rr - r0] = xv;
        dd[rr - r0] = d;
      }
    });
  __syncthreads();
  if (k > 1) {
    if (threadIdx.x == 0) {
      // release at device scope: every x load of this workgroup (ordered
      // before this thread by the barrier above) happens before any write of
      // x by a workgroup that sees this arrival
      const unsigned long long old = __hip_atomic_fetch_add(cnt + it.cnt, 1ull, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
      const unsigned long long target = (old / unsigned(k) + 1) * unsigned(k);
      int good = 1;
      unsigned spins = 0;
      while (__hip_atomic_load(cnt + it.cnt, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
        if (++spins > limit || __hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) {
          atomicExch(err, 1);
          good = 0;
          break;
        }
        __builtin_amdgcn_s_sleep(1);
      }
      // acquire at device scope, paired with the other workgroups' releases
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
      s_ok = good;
    }
    __syncthreads();
    if (!s_ok) return;
  }
  {
    auto ij = [nr, r0](int t, int& i, int& cb) {
      i = r0 + t % nr;
      cb = t / nr;
    };
    auto put = [pp, nr](int t, double v) { pp[(t / nr) * RB + t % nr] = v; };
    if (rec.f32)
      mx_gemv_pairs(a32, rec.fac, rp, n, nr * nb, NT, ij, put);
    else
      mx_gemv_pairs(a64, rec.fac, rp, n, nr * nb, NT, ij, put);
  }
  __syncthreads();
  for (int ii = threadIdx.x; ii < nr; ii += NT) {
    double s = 0.0;
    for (int cb = 0; cb < nb; ++cb) s += pp[cb * RB + ii];
    if (!smask || smask[rec.slot + r0 + ii]) x[dd[ii]] = xo[ii] + alpha * s;
  }
}

typedef __attribute__((address_space(3))) void* lds_ptr_t;

// Direct-to-LDS copy of rows r0 .. r0+63 of every column of a patch inverse
// (column-major, n x n, elements of S bytes at `col0`) into `slice`, column j
// at slice + j * 64 * S bytes. One dword per lane per instruction lands at
// the instruction's LDS base + lane * 4; rows at or past n read the column's
// first element instead (kept in bounds, never used). Waves w0 .. 15 issue
// the instructions round robin; the caller waits (vmcnt) before the slice is
// read. A wave's loads complete in order, so loads issued after the copy wait
// for it too.
template <int S>
__device__ __forceinline__ void mx_prefetch_slice(const unsigned char* __restrict__ col0, int n, int r0,
                                                  unsigned char* slice, int w0) {
  constexpr int PER_COL = 64 * S / 256;   // instructions per column (2 for FP64, 1 for FP32)
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  if (wave < w0) return;
  const int total = n * PER_COL;
  for (int q = wave - w0; q < total; q += 16 - w0) {
    const int j = q / PER_COL, h = q % PER_COL;
    const int dword = h * 64 + lane;                 // dword index inside the column's 64-row slot
    const int row = r0 + dword / (S / 4);
    const int part = dword % (S / 4);
    const int64_t el = int64_t(j) * n + (row < n ? row : 0);
    const unsigned char* g = col0 + el * S + part * 4;
    __builtin_amdgcn_global_load_lds(reinterpret_cast<const void*>(g), (lds_ptr_t)(slice + int64_t(j) * 64 * S + h * 256),
                                     4, 0, 0);
  }
}

// GEMV items of one workgroup's rows from the LDS slice: the same items,
// pairing and arithmetic as mx_gemv_pairs (only the loads differ).
template <typename T, typename IJ, typename Put>
__device__ __forceinline__ void mx_gemv_lds(const T* slice, int r0, const double* __restrict__ rp, int n, int count,
                                            int stride, IJ ij, Put put) {
  for (int t = threadIdx.x; t < count; t += stride) {
    int i, cb;
    ij(t, i, cb);
    const int j0 = cb * MX_CB, w = min(MX_CB, n - j0);
    T m[MX_CB];
#pragma unroll
    for (int jj = 0; jj < MX_CB; ++jj) m[jj] = jj < w ? slice[(j0 + jj) * 64 + (i - r0)] : T(0);
    put(t, mx_dot_item(m, rp, n, cb));
  }
}

// GEMV items of one workgroup's rows read straight from the stored inverse,
// one item at a time (fewer live registers than the paired form): the same
// items and arithmetic as mx_gemv_pairs.
template <typename T, typename IJ, typename Put>
__device__ __forceinline__ void mx_gemv_single(const T* __restrict__ arena, int64_t fac, const double* __restrict__ rp,
                                               int n, int count, int stride, IJ ij, Put put) {
  for (int t = threadIdx.x; t < count; t += stride) {
    int i, cb;
    ij(t, i, cb);
    T m[MX_CB];
    mx_load_item(arena, fac, n, i, cb, true, m);
    put(t, mx_dot_item(m, rp, n, cb));
  }
}

// Cooperative form with a shared residual: as k_mult_coop<64>, but each of
// the k workgroups of a patch forms only its own 64 residual rows and stores
// them to the patch's slots of rbuf with device-coherent stores; after the
// arrival barrier every workgroup reads the whole residual back with
// device-coherent loads. The arrival is a release and the wait ends with an
// acquire, both at device scope, so a workgroup that has seen all k arrivals
// reads the final values, and every workgroup's x loads happen before any x
// write of the patch. Rows, items and block order are those of k_mult_exp, so the
// results equal it bit for bit. Waves 0 .. 7 form the residual without
// waiting for the item record (row records hold everything, including the
// row's place in rbuf); waves 8 .. 15 copy the 64-row slice of the inverse to
// LDS meanwhile, so no residual load queues behind the copy.
__global__ __launch_bounds__(1024) void k_mult_coopr(const CoopItem* __restrict__ items,
                                                     const int4* __restrict__ irow, const double* __restrict__ a64,
                                                     const float* __restrict__ a32, StencilCoef sc,
                                                     const int32_t* __restrict__ ecol, const double* __restrict__ eval,
                                                     const double* __restrict__ b, double* __restrict__ x,
                                                     double alpha, const uint8_t* __restrict__ smask,
                                                     double* __restrict__ rbuf, unsigned long long* __restrict__ cnt,
                                                     int* __restrict__ err, unsigned limit, int pf_bytes) {
  constexpr int NT = 1024, RB = 64;
  extern __shared__ double smem[];
  __shared__ int s_ok;
  // this item's 64 rows (unknown, E_E range, place in the shared residual
  // buffer or -1 for a patch of one item; unknown -1 past the patch) sit at a
  // fixed place: the residual needs nothing from the item record, whose load
  // completes meanwhile
  const int4* rows = irow + int64_t(blockIdx.x) * RB;
  const CoopItem it = items[blockIdx.x];
  // LDS: the prefetched GEMV slice (pf_bytes), this item's pre-update values
  // and unknowns (fixed offsets), then the residual (n rows) and block partials
  unsigned char* slice = reinterpret_cast<unsigned char*>(smem);
  double* xo = smem + pf_bytes / 8;                    // RB values of this item's unknowns before the update
  int32_t* dd = reinterpret_cast<int32_t*>(xo + RB);   // RB unknowns
  double* rp = xo + RB + RB / 2;                       // n residual rows
  // waves 0 .. 7 form the residual (a group of MX_G lanes per row); waves
  // 8 .. 15 copy this workgroup's 64 rows of the inverse to LDS meanwhile. A
  // wave's loads complete in order, so no residual load waits behind the copy
  // or behind the item record the copy needs.
  constexpr int NR = RB * MX_G;   // residual threads
  static_assert(NR % 64 == 0 && NR < NT, "residual and copy waves are disjoint");
  const MultRec rec = it.rec;
  const int sz = rec.f32 ? 4 : 8;
  auto prefetch = [&](int w0) {
    const int n = rec.n;
    if (int64_t(64) * n * sz > pf_bytes) return;
    if (rec.f32)
      mx_prefetch_slice<4>(reinterpret_cast<const unsigned char*>(a32 + rec.fac), n, it.r0, slice, w0);
    else
      mx_prefetch_slice<8>(reinterpret_cast<const unsigned char*>(a64 + rec.fac), n, it.r0, slice, w0);
  };
  if (threadIdx.x < NR) {
    const int grp = threadIdx.x / MX_G, gl = threadIdx.x % MX_G;
    auto src = [rows](int q) { return rows[q]; };
    mx_residual_rows<1>(src, grp, RB, RB, gl, sc, ecol, eval, b, x, [&](int q, double r, int32_t d, double xv, int w) {
      if (w >= 0)
        __hip_atomic_store(rbuf + w, r, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      else
        rp[q] = r;
      xo[q] = xv;
      dd[q] = d;
    });
    __builtin_amdgcn_s_waitcnt(0);   // this wave's residual stores and x loads have completed
  } else {
    prefetch(NR / 64);
  }
  __syncthreads();
  const int n = rec.n;
  const int nb = (n + MX_CB - 1) / MX_CB;
  const int k = (n + RB - 1) / RB;
  const int r0 = it.r0, nr = min(RB, n - r0);
  double* pp = rp + n;               // nb x RB block partials
  const bool pf = int64_t(64) * n * sz <= pf_bytes;
  if (k == 1) {
    __builtin_amdgcn_s_waitcnt(0);   // the slice has landed
    __syncthreads();
  } else {
    unsigned long long old = 0;
    // release at device scope: this workgroup's residual stores (ordered
    // before this thread by the barrier above) are visible to every workgroup
    // that sees the arrival, and its x loads happen before their x writes
    if (threadIdx.x == 0)
      old = __hip_atomic_fetch_add(cnt + it.cnt, 1ull, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    if (threadIdx.x == 0) {
      const unsigned long long target = (old / unsigned(k) + 1) * unsigned(k);
      int good = 1;
      unsigned spins = 0;
      while (__hip_atomic_load(cnt + it.cnt, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
        if (++spins > limit || __hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) {
          atomicExch(err, 1);
          good = 0;
          break;
        }
        __builtin_amdgcn_s_sleep(1);
      }
      // acquire at device scope, paired with the other workgroups' releases
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
      s_ok = good;
    }
    __syncthreads();
    if (!s_ok) {
      __builtin_amdgcn_s_waitcnt(0);   // no copy into LDS outlives the workgroup
      return;
    }
    const double* ra = rbuf + rec.slot;
    for (int j = threadIdx.x; j < n; j += NT) rp[j] = __hip_atomic_load(ra + j, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __builtin_amdgcn_s_waitcnt(0);   // the slice has landed
    __syncthreads();
  }
  {
    auto ij = [nr, r0](int t, int& i, int& cb) {
      i = r0 + t % nr;
      cb = t / nr;
    };
    auto put = [pp, nr](int t, double v) { pp[(t / nr) * RB + t % nr] = v; };
    if (pf) {
      if (rec.f32)
        mx_gemv_lds(reinterpret_cast<const float*>(slice), r0, rp, n, nr * nb, NT, ij, put);
      else
        mx_gemv_lds(reinterpret_cast<const double*>(slice), r0, rp, n, nr * nb, NT, ij, put);
    } else if (rec.f32) {
      mx_gemv_single(a32, rec.fac, rp, n, nr * nb, NT, ij, put);
    } else {
      mx_gemv_single(a64, rec.fac, rp, n, nr * nb, NT, ij, put);
    }
  }
  __syncthreads();
  for (int ii = threadIdx.x; ii < nr; ii += NT) {
    double s = 0.0;
    for (int cb = 0; cb < nb; ++cb) s += pp[cb * RB + ii];
    if (!smask || smask[rec.slot + r0 + ii]) x[dd[ii]] = xo[ii] + alpha * s;
  }
}

// One phase of the multiplicative sweep for a block of kb <= 16 right-hand
// sides (columns of B and X, stride ldv) sharing the level's factors: one
// 1024-thread workgroup per patch. (0) The patch unknowns and their E_E entry
// ranges into LDS. (1) The residual rows of all kb columns into LDS as an
// n x 16 block: a wavefront takes MR_RR rows at once, lane = (column c,
// entry slice e of 4): slice e sums the row's E_E entries e, e + 4, ... for
// column c, slice 0 adds the stencil part, and the four slices are summed by
// lane exchanges. (2) delta = K_p^{-1} R as FP64 MFMA 16x16x4 products, a
// wavefront per 16-row tile, MR_KU loads of the stored inverse issued before
// their products (A operand: row l % 16, column l / 16 of the step; B
// operand: R row l / 16, column l % 16; result row l / 16 + 4 r, column
// l % 16). (3) x += alpha delta at the patch unknowns. Every x read of the
// patch precedes every x write (barrier after (1)); patches of one phase
// share no unknown and no coupling.
typedef double mx_d4 __attribute__((ext_vector_type(4)));
constexpr int MR_CB = 16;   // right-hand sides per block
constexpr int MR_RR = 4;    // residual rows per wavefront at once
constexpr int MR_PER = 4;   // E_E entries a lane loads at once
constexpr int MR_KU = 8;    // MFMA k-steps whose loads are issued together
template <typename T>
__device__ __forceinline__ mx_d4 mr_tile(const T* __restrict__ M, int n, int t0, const double* __restrict__ R,
                                         int lane) {
  const int li = lane % 16, lk = lane / 16, i = t0 + li;
  mx_d4 acc = {0.0, 0.0, 0.0, 0.0};
  const T* col = M + i;
  for (int k0 = 0; k0 < n; k0 += 4 * MR_KU) {
    T a[MR_KU];
#pragma unroll
    for (int u = 0; u < MR_KU; ++u) {
      const int kk = k0 + 4 * u + lk;
      a[u] = (i < n && kk < n) ? col[int64_t(kk) * n] : T(0);
    }
#pragma unroll
    for (int u = 0; u < MR_KU; ++u) {
      const int kk = k0 + 4 * u + lk;
      const double bv = kk < n ? R[kk * MR_CB + li] : 0.0;
      acc = __builtin_amdgcn_mfma_f64_16x16x4f64(double(a[u]), bv, acc, 0, 0, 0);
    }
  }
  return acc;
}

__global__ __launch_bounds__(1024) void k_mult_mrhs(const MultRec* __restrict__ recs, const double* __restrict__ a64,
                                                    const float* __restrict__ a32, const int32_t* __restrict__ slot_dof,
                                                    StencilCoef sc, const int2* __restrict__ slot_q,
                                                    const int32_t* __restrict__ ecol, const double* __restrict__ eval,
                                                    const double* __restrict__ B, double* __restrict__ X, int64_t ldv,
                                                    int kb, double alpha, const uint8_t* __restrict__ smask) {
  extern __shared__ double smem[];
  const MultRec rec = recs[blockIdx.x];
  const int n = rec.n;
  double* R = smem;                                            // n x MR_CB
  int2* ql = reinterpret_cast<int2*>(smem + int64_t(n) * MR_CB);  // E_E entry ranges
  int32_t* dl = reinterpret_cast<int32_t*>(ql + n);             // patch unknowns
  for (int i = threadIdx.x; i < n; i += 1024) {
    dl[i] = slot_dof[rec.slot + i];
    ql[i] = slot_q[rec.slot + i];
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  {
    const int c = lane & 15, e = lane >> 4;
    const bool live = c < kb;
    const double* xc = X + int64_t(c) * ldv;
    for (int r0 = wave * MR_RR; r0 < n; r0 += 16 * MR_RR) {
      int q0[MR_RR], q1[MR_RR];
      double acc[MR_RR], st[MR_RR], bv[MR_RR];
      int rounds = 0;
#pragma unroll
      for (int u = 0; u < MR_RR; ++u) {
        const int rr = r0 + u;
        const int2 q = (rr < n && live) ? ql[rr] : make_int2(0, 0);
        q0[u] = q.x;
        q1[u] = q.y;
        rounds = max(rounds, (q.y - q.x + 4 * MR_PER - 1) / (4 * MR_PER));
        const bool own = rr < n && live && e == 0;
        st[u] = own ? krow(dl[rr], xc, sc, nullptr, nullptr, nullptr) : 0.0;
        bv[u] = own ? B[int64_t(c) * ldv + dl[rr]] : 0.0;
        acc[u] = 0.0;
      }
      for (int k0 = 0; k0 < rounds; ++k0) {
        int ci[MR_RR][MR_PER];
        double cv[MR_RR][MR_PER], xv[MR_RR][MR_PER];
#pragma unroll
        for (int u = 0; u < MR_RR; ++u)
#pragma unroll
          for (int k = 0; k < MR_PER; ++k) {
            const int q = q0[u] + k0 * 4 * MR_PER + e + 4 * k;
            ci[u][k] = q < q1[u] ? ecol[q] : -1;
            cv[u][k] = q < q1[u] ? eval[q] : 0.0;
          }
#pragma unroll
        for (int u = 0; u < MR_RR; ++u)
#pragma unroll
          for (int k = 0; k < MR_PER; ++k) xv[u][k] = ci[u][k] >= 0 ? xc[ci[u][k]] : 0.0;
#pragma unroll
        for (int u = 0; u < MR_RR; ++u)
#pragma unroll
          for (int k = 0; k < MR_PER; ++k) acc[u] += cv[u][k] * xv[u][k];
      }
#pragma unroll
      for (int u = 0; u < MR_RR; ++u) {
        double v = acc[u] + st[u];
        v += __shfl_xor(v, 16);
        v += __shfl_xor(v, 32);
        const int rr = r0 + u;
        if (e == 0 && rr < n) R[rr * MR_CB + c] = live ? bv[u] - v : 0.0;
      }
    }
  }
  __syncthreads();
  const int li = lane % 16, lk = lane / 16;
  for (int t0 = wave * 16; t0 < n; t0 += 256) {
    const mx_d4 acc = rec.f32 ? mr_tile(a32 + rec.fac, n, t0, R, lane) : mr_tile(a64 + rec.fac, n, t0, R, lane);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = t0 + lk + 4 * r;
      if (row < n && li < kb && (!smask || smask[rec.slot + row])) X[int64_t(li) * ldv + dl[row]] += alpha * acc[r];
    }
  }
}

// One colour phase of the shared standard patches: cells with
// (i + 3 j) mod 8 == colour and no E_E entries solve their 5x5 patch from the
// current residual and update x.
__device__ __forceinline__ void std_cell(int N, int colour, int64_t t, const uint8_t* __restrict__ flag,
                                         const double* __restrict__ Minv, StencilCoef sc,
                                         const double* __restrict__ b, double* __restrict__ x, double alpha) {
  // cells of one colour in row i: j = 3 (colour - i) mod 8 + 8 m (3 is its own
  // inverse mod 8); consecutive threads take consecutive m, 64 bytes apart
  const int per = N / 8;
  const int i = int(t / per), m = int(t % per);
  const int j = ((3 * (colour - i)) % 8 + 8) % 8 + 8 * m;
  const int64_t n2 = int64_t(N) * N;
  const int64_t c = int64_t(i) * N + j;
  // the cell's flag loads beside the gathers (a cell with E_E entries is
  // computed too and not written), so the gathers do not wait for it
  const uint8_t fl = flag[c];
  const int ip = wrapi(i + 1, N), jp = wrapi(j + 1, N);
  const int64_t d[5] = {c, int64_t(ip) * N + j, n2 + c, n2 + int64_t(i) * N + jp, 2 * n2 + c};
  const int kind[5] = {0, 0, 1, 1, 2}, ci[5] = {i, ip, i, i, i}, cj[5] = {j, j, j, jp, j};
  double r[5], xv[5];
#pragma unroll
  for (int q = 0; q < 5; ++q) {
    r[q] = b[d[q]] - krow_at(kind[q], ci[q], cj[q], x, sc);
    xv[q] = x[d[q]];
  }
  double dl[5];
#pragma unroll
  for (int q = 0; q < 5; ++q) {
    double s = 0.0;
#pragma unroll
    for (int m = 0; m < 5; ++m) s += Minv[q + 5 * m] * r[m];
    dl[q] = s;
  }
  // an empty statement that takes the updates and old values as inputs: the
  // compiler must form them (and so issue every load) before it branches on
  // the flag
  asm volatile("" ::"v"(dl[0]), "v"(dl[1]), "v"(dl[2]), "v"(dl[3]), "v"(dl[4]), "v"(xv[0]), "v"(xv[1]), "v"(xv[2]),
               "v"(xv[3]), "v"(xv[4]));
  if (fl & 1) return;
#pragma unroll
  for (int q = 0; q < 5; ++q) x[d[q]] = xv[q] + alpha * dl[q];
}

__global__ __launch_bounds__(TPB) void k_mult_std(int N, int colour, const uint8_t* __restrict__ flag,
                                                  const double* __restrict__ Minv, StencilCoef sc,
                                                  const double* __restrict__ b, double* __restrict__ x, double alpha) {
  const int64_t t = int64_t(blockIdx.x) * TPB + threadIdx.x;
  if (t >= int64_t(N) * (N / 8)) return;
  std_cell(N, colour, t, flag, Minv, sc, b, x, alpha);
}

// Grid-wide barrier of the persistent sweep: every workgroup adds one to a
// device counter and waits until it reaches `target` (gridDim.x per barrier
// so far). Release and acquire fences at device scope make the phase's x
// updates visible to every workgroup. The wait is bounded: after `limit`
// polls, or once another workgroup has reported a timeout, the workgroup
// records the failure and returns false, and the kernel stops.
__device__ bool grid_sync(unsigned long long* __restrict__ bar, unsigned long long target, int* __restrict__ err,
                          unsigned limit) {
  __shared__ int ok;
  __syncthreads();
  if (threadIdx.x == 0) {
    __threadfence();
    atomicAdd(bar, 1ull);
    int good = 1;
    unsigned spins = 0;
    while (__hip_atomic_load(bar, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) < target) {
      if (__hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0 || ++spins > limit) {
        atomicExch(err, 1);
        good = 0;
        break;
      }
      __builtin_amdgcn_s_sleep(2);
    }
    __threadfence();
    ok = good;
  }
  __syncthreads();
  return ok != 0;
}

struct SweepArgs {
  const MultRec* recs;
  const int32_t* ph_ptr;   // device copy of the phase offsets
  int nph;
  const double* a64;
  const float* a32;
  const int32_t* slot_dof;
  StencilCoef sc;
  const int2* slot_q;
  const int32_t* ecol;
  const double* eval;
  const uint8_t* flag;
  const double* std_inv;
  const double* b;
  double* x;
  double alpha;
  unsigned long long* bar;
  int* err;
  unsigned limit;
  int std_first;           // shared-patch colours before the explicit phases
  const uint8_t* smask;    // injection mask of the box family, or nullptr
};

// The whole multiplicative sweep of one level in one cooperative launch: the
// explicit colour phases (patches of a phase spread over the workgroups, each
// processed exactly as by k_mult_exp), then the 8 colours of shared standard
// patches (each cell exactly as by k_mult_std), a grid barrier after each
// phase. Same arithmetic, same order of phases: bit-identical to the
// per-phase launches.
template <int NT>
__global__ __launch_bounds__(NT) void k_mult_sweep(SweepArgs a) {
  extern __shared__ double smem[];
  const unsigned long long G = gridDim.x;
  unsigned long long target = 0;
  const int N = a.sc.N;
  const int64_t total = int64_t(N) * (N / 8);
  // stage 0: explicit colour phases; stage 1: shared-patch colours (order swapped by std_first)
  for (int stage = 0; stage < 2; ++stage) {
    const bool explicit_stage = (stage == 0) != (a.std_first != 0);
    if (explicit_stage) {
      for (int ph = 0; ph < a.nph; ++ph) {
        const int p1 = a.ph_ptr[ph + 1];
        for (int p = a.ph_ptr[ph] + int(blockIdx.x); p < p1; p += int(G)) {
          const MultRec rec = a.recs[p];
          mx_patch<NT>(rec, smem, a.a64, a.a32, a.slot_dof, a.sc, a.slot_q, a.ecol, a.eval, a.b, a.x, a.alpha,
                       a.smask);
          __syncthreads();
        }
        if (stage == 1 && ph == a.nph - 1) break;
        target += G;
        if (!grid_sync(a.bar, target, a.err, a.limit)) return;
      }
    } else {
      for (int col = 0; col < 8; ++col) {
        for (int64_t t = int64_t(blockIdx.x) * NT + threadIdx.x; t < total; t += int64_t(G) * NT)
          std_cell(N, col, t, a.flag, a.std_inv, a.sc, a.b, a.x, a.alpha);
        if (stage == 1 && col == 7) break;
        target += G;
        if (!grid_sync(a.bar, target, a.err, a.limit)) return;
      }
    }
  }
}

// ---- dataflow form of a level's explicit-patch sweep ----
// One launch runs every explicit phase of a sweep. Work items are the
// (patch, 64-row block) items of the shared-residual form in phase order; a
// workgroup claims the next item from a ticket counter, and an item of patch
// p starts its residual only when every patch of an earlier colour that
// conflicts with p (shares an unknown or a K_E coupling) has finished this
// sweep: each finished item adds one to the arrival counter of every
// successor of its patch (after a release fence at device scope), and p
// waits, on one counter with one lane, for the number of items of all its
// predecessors. Non-conflicting patches commute, so the result equals the
// sweep in phase order bit for bit, while independent regions of the
// structure run through their colours without waiting for each other and no
// phase waits for a launch. Before that wait the item's row records, E_E
// entries, b and its 64-row slice of the inverse are already loaded.
// Progress: items are claimed in order and an item waits only on items of
// smaller index, all claimed by running workgroups, so the smallest unfinished
// item can always proceed. Every wait is bounded (a timeout sets err; then
// every workgroup stops claiming and the host reports the failure).
// Counters are monotonic: the ticket is `base` plus items claimed, and the
// arrival counter of patch p reaches `sweep` times its wait count when every
// predecessor has finished this sweep.
struct FlowArgs {
  const CoopItem* items;
  const int4* irow;
  int64_t n_items;
  const double* a64;
  const float* a32;
  StencilCoef sc;
  const int32_t* ecol;
  const double* eval;
  const double* b;
  double* x;
  double alpha;
  const uint8_t* smask;
  double* rbuf;
  unsigned long long* pcnt;     // arrival counters of the 64-row items of each patch
  unsigned long long* flow;     // [0] ticket, [1 + p] completions signalled to patch p
  unsigned long long base, sweep;
  const int32_t* succ_ptr;      // phase-order patch -> successor range (n + 1), then its wait count (n)
  const int32_t* succ;          // successors
  int32_t n_rec;                // patches
  int* err;
  unsigned limit;
  int pf_bytes;
};

// One lane waits until *ctr >= target (bounded); false on a timeout (err set)
// or when another workgroup has reported one.
__device__ __forceinline__ bool flow_wait(const unsigned long long* ctr, unsigned long long target, int* err,
                                          unsigned limit) {
  unsigned spins = 0;
  while (__hip_atomic_load(ctr, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
    if (++spins > limit) {
      atomicExch(err, 1);
      return false;
    }
    if ((spins & 63) == 0 && __hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) return false;
    __builtin_amdgcn_s_sleep(1);
  }
  return true;
}

__global__ __launch_bounds__(1024) void k_mult_flow(FlowArgs a) {
  constexpr int NT = 1024, RB = 64;
  constexpr int NR = RB * MX_G;            // waves 0 .. 7 form the residual rows
  constexpr int POLL_WAVE = NR / 64;       // wave 8 waits for the predecessors
  constexpr int COPY_W0 = POLL_WAVE + 1;   // waves 9 .. 15 copy the inverse slice
  static_assert(COPY_W0 < NT / 64, "copy waves exist");
  extern __shared__ double smem[];
  __shared__ int s_t, s_ok;
  unsigned char* slice = reinterpret_cast<unsigned char*>(smem);
  double* xo = smem + a.pf_bytes / 8;                  // RB values of this item's unknowns before the update
  int32_t* dd = reinterpret_cast<int32_t*>(xo + RB);   // RB unknowns
  double* rp = xo + RB + RB / 2;                       // n residual rows, then the block partials
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int grp = threadIdx.x / MX_G, gl = threadIdx.x % MX_G;
  for (;;) {
    if (threadIdx.x == 0) {
      int t = -1;
      if (__hip_atomic_load(a.err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0) {
        const unsigned long long q =
            __hip_atomic_fetch_add(a.flow, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) - a.base;
        if (q < static_cast<unsigned long long>(a.n_items)) t = int(q);
      }
      s_t = t;
      s_ok = 1;
    }
    __syncthreads();
    const int t = s_t;
    if (t < 0) return;
    const CoopItem it = a.items[t];
    const MultRec rec = it.rec;
    const int n = rec.n, k = (n + RB - 1) / RB, r0 = it.r0, nr = min(RB, n - r0);
    const int p = it.cnt;
    const int sz = rec.f32 ? 4 : 8;
    const bool pf = int64_t(64) * n * sz <= a.pf_bytes;
    // (1) before the wait: row records, the first round of E_E entries and b
    // (residual waves), the predecessor wait (poll wave), the slice (copy waves)
    int d = -1, q0 = 0, q1 = 0, qw = -1;
    double bv = 0.0;
    int cidx[MX_PER];
    double cv[MX_PER];
    if (threadIdx.x < NR) {
      const int4 q = a.irow[int64_t(t) * RB + grp];
      d = q.x;
      q0 = q.y;
      q1 = q.z;
      qw = q.w;
      bv = (gl == 0 && d >= 0) ? a.b[d] : 0.0;
#pragma unroll
      for (int kk = 0; kk < MX_PER; ++kk) {
        const int e = q0 + gl + MX_G * kk;
        cidx[kk] = e < q1 ? a.ecol[e] : -1;
        cv[kk] = e < q1 ? a.eval[e] : 0.0;
      }
    } else if (wave == POLL_WAVE) {
      if (lane == 0) {
        const unsigned long long need = static_cast<unsigned long long>(a.succ_ptr[a.n_rec + 1 + p]);
        if (!flow_wait(a.flow + 1 + p, a.sweep * need, a.err, a.limit)) s_ok = 0;
      }
      // acquire at device scope, paired with every predecessor's release
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    } else if (pf) {
      if (rec.f32)
        mx_prefetch_slice<4>(reinterpret_cast<const unsigned char*>(a.a32 + rec.fac), n, r0, slice, COPY_W0);
      else
        mx_prefetch_slice<8>(reinterpret_cast<const unsigned char*>(a.a64 + rec.fac), n, r0, slice, COPY_W0);
    }
    __syncthreads();
    if (!s_ok) {
      __builtin_amdgcn_s_waitcnt(0);   // no copy into LDS outlives the workgroup
      return;
    }
    // (2) residual rows (the arithmetic of mx_residual_rows, row by row)
    if (threadIdx.x < NR) {
      const bool own = gl == 0 && d >= 0;
      const double stv = own ? krow(d, a.x, a.sc, nullptr, nullptr, nullptr) : 0.0;
      const double xd = own ? a.x[d] : 0.0;
      double xv[MX_PER];
#pragma unroll
      for (int kk = 0; kk < MX_PER; ++kk) xv[kk] = cidx[kk] >= 0 ? a.x[cidx[kk]] : 0.0;
      double acc = 0.0;
      if (q0 < q1) {
#pragma unroll
        for (int kk = 0; kk < MX_PER; ++kk) acc += cv[kk] * xv[kk];
      }
      const int rounds = (q1 - q0 + MX_G * MX_PER - 1) / (MX_G * MX_PER);
      for (int k0 = 1; k0 < rounds; ++k0) {
        int ci[MX_PER];
        double cw[MX_PER], xw[MX_PER];
#pragma unroll
        for (int kk = 0; kk < MX_PER; ++kk) {
          const int e = q0 + k0 * MX_G * MX_PER + gl + MX_G * kk;
          ci[kk] = e < q1 ? a.ecol[e] : -1;
          cw[kk] = e < q1 ? a.eval[e] : 0.0;
        }
#pragma unroll
        for (int kk = 0; kk < MX_PER; ++kk) xw[kk] = ci[kk] >= 0 ? a.x[ci[kk]] : 0.0;
#pragma unroll
        for (int kk = 0; kk < MX_PER; ++kk) acc += cw[kk] * xw[kk];
      }
      if (own) acc += stv;
#pragma unroll
      for (int o = MX_G / 2; o > 0; o >>= 1) acc += __shfl_down(acc, o, MX_G);
      if (own) {
        const double r = bv - acc;
        if (qw >= 0)
          __hip_atomic_store(a.rbuf + qw, r, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        else
          rp[grp] = r;
        xo[grp] = xd;
        dd[grp] = d;
      }
      __builtin_amdgcn_s_waitcnt(0);   // this wave's residual stores and x loads have completed
    }
    __syncthreads();
    // (3) a patch over several items: exchange the residual rows
    if (k > 1) {
      if (threadIdx.x == 0) {
        const unsigned long long old =
            __hip_atomic_fetch_add(a.pcnt + p, 1ull, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        const unsigned long long target = (old / unsigned(k) + 1) * unsigned(k);
        const bool ok = flow_wait(a.pcnt + p, target, a.err, a.limit);
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        s_ok = ok ? 1 : 0;
      }
      __syncthreads();
      if (!s_ok) {
        __builtin_amdgcn_s_waitcnt(0);
        return;
      }
      const double* ra = a.rbuf + rec.slot;
      for (int j = threadIdx.x; j < n; j += NT) rp[j] = __hip_atomic_load(ra + j, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    __builtin_amdgcn_s_waitcnt(0);   // the slice has landed
    __syncthreads();
    // (4) this item's rows of delta = K_p^{-1} r (items and block order of k_mult_exp)
    const int nb = (n + MX_CB - 1) / MX_CB;
    double* pp = rp + n;
    {
      auto ij = [nr, r0](int q, int& i, int& cb) {
        i = r0 + q % nr;
        cb = q / nr;
      };
      auto put = [pp, nr](int q, double v) { pp[(q / nr) * RB + q % nr] = v; };
      if (pf) {
        if (rec.f32)
          mx_gemv_lds(reinterpret_cast<const float*>(slice), r0, rp, n, nr * nb, NT, ij, put);
        else
          mx_gemv_lds(reinterpret_cast<const double*>(slice), r0, rp, n, nr * nb, NT, ij, put);
      } else if (rec.f32) {
        mx_gemv_single(a.a32, rec.fac, rp, n, nr * nb, NT, ij, put);
      } else {
        mx_gemv_single(a.a64, rec.fac, rp, n, nr * nb, NT, ij, put);
      }
    }
    __syncthreads();
    // (5) x at this item's rows, then the done count (release at device scope)
    for (int ii = threadIdx.x; ii < nr; ii += NT) {
      double sacc = 0.0;
      for (int cb = 0; cb < nb; ++cb) sacc += pp[cb * RB + ii];
      if (!a.smask || a.smask[rec.slot + r0 + ii])
        __hip_atomic_store(a.x + dd[ii], xo[ii] + a.alpha * sacc, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    __builtin_amdgcn_s_waitcnt(0);   // every wave's x stores have completed
    __syncthreads();
    // signal every successor: release at device scope, then one arrival each
    if (wave == 0) {
      const int sa = a.succ_ptr[p], sb = a.succ_ptr[p + 1];
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
      for (int i = sa + lane; i < sb; i += 64)
        __hip_atomic_fetch_add(a.flow + 1 + a.succ[i], 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
  }
}

__global__ void k_zero_u64(unsigned long long* v, int64_t n) {
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t < n) v[t] = 0ull;
}

__global__ void k_zero_bar(unsigned long long* bar, int words) {
  if (blockIdx.x == 0 && int(threadIdx.x) < words) bar[threadIdx.x] = 0ull;
}

}  // namespace

// Workgroups of the cooperative sweep of level L (0: not possible).
static int sweep_grid(const Level& L) {
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void*>(k_mult_sweep<1024>), 1024,
                                                   L.mx_lds) != hipSuccess)
    return 0;
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) !=
                                              hipSuccess)
    return 0;
  const int cap = per_cu * cus;
  int want = int((int64_t(L.N) * (L.N / 8) + 1023) / 1024);
  for (size_t ph = 0; ph + 1 < L.ph_ptr.size(); ++ph) want = std::max(want, L.ph_ptr[ph + 1] - L.ph_ptr[ph]);
  return std::min(cap, std::max(want, 1));
}

void launch_clear_sweep_flags(Ctx& c, hipStream_t s) {
  if (c.d_bar) k_zero_bar<<<1, 64, 0, s>>>(c.d_bar, 2);
}

bool launch_mult_sweep(Ctx& c, Level& L, const double* b, double* x, hipStream_t s) {
  const int nph = int(L.ph_ptr.size()) - 1;
  if (nph <= 0 || !L.d_ph_ptr || !c.d_bar) return false;
  if (L.sweep_grid == 0) L.sweep_grid = sweep_grid(L);
  if (L.sweep_grid <= 0) return false;
  SweepArgs a{L.d_mrec, L.d_ph_ptr, nph, L.d_f64, L.d_f32, L.d_slot_dof, L.sc, L.d_slot_q, L.d_ecol, L.d_eval,
              L.d_cellflag, L.d_std_inv, b, x, level_alpha(c, L), c.d_bar, reinterpret_cast<int*>(c.d_bar + 1),
              c.wait_limit, c.std_first ? 1 : 0, L.d_slot_mask};
  k_zero_bar<<<1, 64, 0, s>>>(c.d_bar, 1);
  double bytes = 0.0;
  for (double v : L.ph_bytes) bytes += v;
  timing_begin(c, s);
  void* args[] = {&a};
  CAV_HIP(hipLaunchCooperativeKernel(reinterpret_cast<const void*>(k_mult_sweep<1024>), dim3(L.sweep_grid),
                                     dim3(1024), args, L.mx_lds, s));
  timing_end(c, s, bytes, nph);
  return true;
}

void launch_zero_u64(unsigned long long* v, int64_t n, hipStream_t s) {
  if (n > 0) k_zero_u64<<<unsigned((n + 255) / 256), 256, 0, s>>>(v, n);
}

// Workgroups of the dataflow sweep of level L: as many as stay resident (one
// item each at a time), at most one per item; 0 if not possible.
static int flow_grid(const Level& L) {
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void*>(k_mult_flow), 1024,
                                                   L.cr_lds) != hipSuccess)
    return 0;
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) !=
                                              hipSuccess)
    return 0;
  const int grid = int(std::min<int64_t>(int64_t(per_cu) * cus, L.flow_items));
  // the items of one patch meet at a barrier: all of them must be claimable at once
  const int k_max = (std::max<int32_t>(L.mrec_max_n, 1) + 63) / 64;
  return grid >= std::min<int64_t>(k_max, L.flow_items) ? grid : 0;
}

bool launch_mult_flow(Ctx& c, Level& L, const double* b, double* x, hipStream_t s) {
  if (c.capturing || L.flow_items <= 0 || !L.d_flow || !L.d_pr || !L.d_pr_ptr || !L.d_irow || !L.d_citem[0] ||
      !L.d_pcnt || !L.d_delta || !c.d_bar)
    return false;
  if (L.flow_grid == 0) L.flow_grid = flow_grid(L);
  if (L.flow_grid <= 0) return false;
  ++L.flow_sweep;
  FlowArgs a{L.d_citem[0], L.d_irow, L.flow_items, L.d_f64, L.d_f32, L.sc, L.d_ecol, L.d_eval, b, x,
             level_alpha(c, L), L.d_slot_mask, L.d_delta, L.d_pcnt, L.d_flow, L.flow_base, L.flow_sweep,
             L.d_pr_ptr, L.d_pr, int32_t(L.ph_exp.size()), reinterpret_cast<int*>(c.d_bar + 1), c.wait_limit,
             L.cr_pf};
  timing_begin(c, s, 3);
  k_mult_flow<<<unsigned(L.flow_grid), 1024, L.cr_lds, s>>>(a);
  timing_end(c, s, L.flow_bytes, 1);
  // every workgroup ends with one claim past the last item
  L.flow_base += uint64_t(L.flow_items) + uint64_t(L.flow_grid);
  return true;
}

// Zeroes every level's arrival and dataflow counters (after a wait gave up,
// when their counts no longer follow whole rounds).
void reset_sweep_counters(Ctx& c, hipStream_t s) {
  for (Level& L : c.lv) {
    const int64_t nrec = std::max<int64_t>(int64_t(L.ph_exp.size()), 1);
    if (L.d_pcnt) launch_zero_u64(L.d_pcnt, 2 * nrec, s);
    if (L.d_flow) launch_zero_u64(L.d_flow, 1 + nrec, s);
    L.flow_base = L.flow_sweep = 0;
  }
}

// The form a phase launch takes: the cooperative form waits on other
// workgroups of its launch, so inside a captured graph (batched systems run
// concurrently) the one-workgroup form runs instead, with the same results.
static int phase_form(const Ctx& c, const Level& L, int nt) {
  if (nt == 3 && (c.capturing || !c.d_bar || !L.d_pcnt || !L.d_citem[0] || !L.d_irow || !L.d_delta)) return 1024;
  if ((nt == 1 || nt == 2) && (c.capturing || !c.d_bar || !L.d_pcnt || !L.d_citem[nt - 1])) return 1024;
  return nt;
}

void launch_mult_smoother(Ctx& c, Level& L, const double* b, double* x, bool zero_guess, hipStream_t s,
                          bool remove_mean) {
  require_full_layout(L);
  const int64_t n2 = int64_t(L.N) * L.N, n = 3 * n2;
  if (zero_guess) launch_fill(x, 0.0, n, s);
  const int nph = int(L.ph_ptr.size()) - 1;
  if (L.sweep_mode == 1 && !c.capturing && launch_mult_sweep(c, L, b, x, s)) {
    if (remove_mean) launch_pressure_mean_remove(x, L.N, L.d_part, s);
    return;
  }
  const int64_t per_colour = n2 / 8;
  auto standard = [&]() {
    for (int col = 0; col < 8; ++col)
      k_mult_std<<<nblocks(per_colour), TPB, 0, s>>>(L.N, col, L.d_cellflag, L.d_std_inv, L.sc, b, x,
                                                     level_alpha(c, L));
  };
  if (c.std_first) standard();
  if (nph > 0 && !(L.sweep_mode == 2 && launch_mult_flow(c, L, b, x, s))) {
    // one bracket around each run of phase launches of one kernel form
    int open = -1, cnt = 0;
    double bytes = 0.0;
    for (int ph = 0; ph < nph; ++ph) {
      const int nt = phase_form(c, L, L.mx_nt[mx_bucket(L.ph_maxn[ph])]);
      const int kind = nt == 3 ? 2 : (nt == 1 || nt == 2) ? 1 : 0;   // shared residual / cooperative / other
      if (kind != open) {
        if (open >= 0) timing_end(c, s, bytes, cnt);
        timing_begin(c, s, kind);
        open = kind;
        cnt = 0;
        bytes = 0.0;
      }
      launch_mult_phase(c, L, ph, nt, b, x, s);
      bytes += L.ph_bytes[ph];
      ++cnt;
    }
    timing_end(c, s, bytes, cnt);
  }
  if (!c.std_first) standard();
  if (remove_mean) launch_pressure_mean_remove(x, L.N, L.d_part, s);
}

void launch_mult_phase(Ctx& c, Level& L, int ph, int nt, const double* b, double* x, hipStream_t s) {
  require_full_layout(L);
  const int a = L.ph_ptr[ph], cnt = L.ph_ptr[ph + 1] - a;
  const unsigned g = unsigned(cnt);
  nt = phase_form(c, L, nt);
  if (nt == 3) {
    const int w0 = L.ph_wptr[ph], nw = L.ph_wptr[ph + 1] - w0;
    k_mult_coopr<<<unsigned(nw), 1024, L.cr_lds, s>>>(L.d_citem[0] + w0, L.d_irow + int64_t(w0) * 64, L.d_f64,
                                                         L.d_f32, L.sc, L.d_ecol, L.d_eval, b, x, level_alpha(c, L),
                                                         L.d_slot_mask, L.d_delta, L.d_pcnt,
                                                         reinterpret_cast<int*>(c.d_bar + 1), c.wait_limit, L.cr_pf);
    return;
  }
  if (nt == 1 || nt == 2) {
    int* err = reinterpret_cast<int*>(c.d_bar + 1);
    const double al = level_alpha(c, L);
    if (nt == 1) {
      const int w0 = L.ph_wptr[ph], nw = L.ph_wptr[ph + 1] - w0;
      k_mult_coop<64><<<unsigned(nw), 1024, L.cp_lds[0], s>>>(L.d_citem[0] + w0, L.d_f64, L.d_f32, L.d_slot_dof, L.sc,
                                                              L.d_slot_q, L.d_ecol, L.d_eval, b, x, al, L.d_slot_mask,
                                                              L.d_pcnt, err, c.wait_limit);
    } else {
      const int w0 = L.ph_wptr2[ph], nw = L.ph_wptr2[ph + 1] - w0;
      k_mult_coop<128><<<unsigned(nw), 1024, L.cp_lds[1], s>>>(L.d_citem[1] + w0, L.d_f64, L.d_f32, L.d_slot_dof,
                                                               L.sc, L.d_slot_q, L.d_ecol, L.d_eval, b, x, al,
                                                               L.d_slot_mask, L.d_pcnt, err, c.wait_limit);
    }
    return;
  }
  if (nt == 0) {
    const int w0 = L.ph_wptr[ph], nw = L.ph_wptr[ph + 1] - w0;
    k_mult_res<<<unsigned(nw), 256, 0, s>>>(L.d_wrk + w0, L.d_mrec, L.d_slot_dof, L.sc, L.d_slot_q, L.d_ecol,
                                            L.d_eval, b, x, L.d_delta);
    k_mult_gemv<<<unsigned(nw), 256, L.sp_lds, s>>>(L.d_wrk + w0, L.d_mrec, L.d_f64, L.d_f32, L.d_slot_dof,
                                                    L.d_delta, x, level_alpha(c, L), L.d_slot_mask);
    return;
  }
  switch (nt) {
    case 256:
      k_mult_exp<256><<<g, 256, L.mx_lds, s>>>(L.d_mrec + a, L.d_f64, L.d_f32, L.d_slot_dof, L.sc, L.d_slot_q,
                                               L.d_ecol, L.d_eval, b, x, level_alpha(c, L), L.d_slot_mask);
      break;
    case 512:
      k_mult_exp<512><<<g, 512, L.mx_lds, s>>>(L.d_mrec + a, L.d_f64, L.d_f32, L.d_slot_dof, L.sc, L.d_slot_q,
                                               L.d_ecol, L.d_eval, b, x, level_alpha(c, L), L.d_slot_mask);
      break;
    default:
      k_mult_exp<1024><<<g, 1024, L.mx_lds, s>>>(L.d_mrec + a, L.d_f64, L.d_f32, L.d_slot_dof, L.sc, L.d_slot_q,
                                                 L.d_ecol, L.d_eval, b, x, level_alpha(c, L), L.d_slot_mask);
  }
}

// Raises the phase kernel's dynamic-LDS limit once (at setup, never inside a
// launch sequence that may be captured into a graph).
void prepare_mult_smoother(size_t lds) {
  static size_t set_to = 64 * 1024;
  if (lds <= set_to) return;
  for (const void* f : {reinterpret_cast<const void*>(k_mult_exp<256>), reinterpret_cast<const void*>(k_mult_exp<512>),
                        reinterpret_cast<const void*>(k_mult_exp<1024>), reinterpret_cast<const void*>(k_mult_gemv),
                        reinterpret_cast<const void*>(k_mult_sweep<1024>), reinterpret_cast<const void*>(k_mult_coop<64>),
                        reinterpret_cast<const void*>(k_mult_coop<128>), reinterpret_cast<const void*>(k_mult_coopr),
                        reinterpret_cast<const void*>(k_mult_flow),
                        reinterpret_cast<const void*>(k_mult_mrhs)})
    CAV_HIP(hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, int(lds)));
  set_to = lds;
}

// The smoother for a block of kb <= 16 right-hand sides (columns of b and x,
// stride ldv). Multiplicative: every explicit phase in one multi-column
// launch (MFMA), the shared-patch colours and the mean removal per column, in
// the single-column order. Additive: the single-column sweep per column.
void launch_smoother_multi(Ctx& c, Level& L, const double* b, double* x, int64_t ldv, int kb, bool zero_guess,
                           hipStream_t s, bool remove_mean) {
  const int64_t n2 = int64_t(L.N) * L.N, n = 3 * n2;
  if (level_smoother(c, L) != CAV_SMOOTHER_MULTIPLICATIVE) {
    for (int q = 0; q < kb; ++q) launch_smoother(c, L, b + q * ldv, x + q * ldv, zero_guess, s, remove_mean);
    return;
  }
  require_full_layout(L);
  if (zero_guess)
    for (int q = 0; q < kb; ++q) launch_fill(x + q * ldv, 0.0, n, s);
  const int nph = int(L.ph_ptr.size()) - 1;
  const int64_t per_colour = n2 / 8;
  const double al = level_alpha(c, L);
  auto standard = [&]() {
    for (int col = 0; col < 8; ++col)
      for (int q = 0; q < kb; ++q)
        k_mult_std<<<nblocks(per_colour), TPB, 0, s>>>(L.N, col, L.d_cellflag, L.d_std_inv, L.sc, b + q * ldv,
                                                       x + q * ldv, al);
  };
  if (c.std_first) standard();
  for (int ph = 0; ph < nph; ++ph) {
    const int a = L.ph_ptr[ph], cnt = L.ph_ptr[ph + 1] - a;
    k_mult_mrhs<<<unsigned(cnt), 1024, L.mr_lds, s>>>(L.d_mrec + a, L.d_f64, L.d_f32, L.d_slot_dof, L.sc, L.d_slot_q,
                                                     L.d_ecol, L.d_eval, b, x, ldv, kb, al, L.d_slot_mask);
  }
  if (!c.std_first) standard();
  if (remove_mean)
    for (int q = 0; q < kb; ++q) launch_pressure_mean_remove(x + q * ldv, L.N, L.d_part, s);
}

void launch_smoother(Ctx& c, Level& L, const double* b, double* x, bool zero_guess, hipStream_t s,
                     bool remove_mean) {
  if (level_smoother(c, L) == CAV_SMOOTHER_MULTIPLICATIVE) {
    launch_mult_smoother(c, L, b, x, zero_guess, s, remove_mean);
    return;
  }
  const int64_t n2 = int64_t(L.N) * L.N;
  const double* r = b;
  if (!zero_guess) {
    launch_apply_op(L, x, L.d_r, b, s);  // r = b - K x
    r = L.d_r;
  }
  const int p64 = int(L.rec64_h.size()), p32 = int(L.rec32_h.size());
  int maxn = 0;
  if (p64) maxn = L.rec64_h[0].n;
  if (p32) maxn = std::max(maxn, L.rec32_h[0].n);
  // LDS: the gathered residual and either the column-group partials or the
  // symmetric form's direct (64 per item) and mirrored (16 per item) partials
  const size_t lds = L.packed ? (size_t(maxn) + 2 + size_t(sym_items(maxn)) * 80) * sizeof(double)
                              : (size_t(maxn) + 2 + AS_THREADS) * sizeof(double);
  const unsigned grid = unsigned(p64 + p32) + unsigned((n2 + AS_THREADS - 1) / AS_THREADS);
  const double al = level_alpha(c, L);
  // factors beyond the 256 MB last-level cache are streamed (read once per
  // sweep); smaller levels keep theirs cached between sweeps
  const bool stream = L.bytes64 + L.bytes32 > 256e6;
  auto go = [&](auto kern) {
    kern<<<grid, AS_THREADS, lds, s>>>(p64, L.d_rec64, L.d_f64, p32, L.d_rec32, L.d_f32, L.d_slot_dof, L.d_delta, L.N,
                                       L.d_cellflag, L.d_std_inv, r, L.d_z, x, al, zero_guess ? 1 : 0);
  };
  timing_begin(c, s);
  if (L.packed)
    stream ? go(k_add_smooth<true, true>) : go(k_add_smooth<false, true>);
  else
    stream ? go(k_add_smooth<true, false>) : go(k_add_smooth<false, false>);
  timing_end(c, s, L.bytes64 + L.bytes32 + 72.0 * double(n2));
  if (L.n_touched > 0) {
    const double per = double(L.n_slots) / double(L.n_touched);
    auto go_t = [&](auto kern, int lanes) {
      kern<<<nblocks(int64_t(L.n_touched) * lanes), TPB, 0, s>>>(L.n_touched, L.d_t_dof, L.d_t_inv, L.d_t_ptr,
                                                                L.d_t_slot, L.d_delta, L.d_z, x, al, zero_guess ? 1 : 0);
    };
    if (per <= 12.0) go_t(k_touched<8>, 8);
    else if (per <= 24.0) go_t(k_touched<16>, 16);
    else if (per <= 48.0) go_t(k_touched<32>, 32);
    else go_t(k_touched<64>, 64);
  }
  if (remove_mean) launch_pressure_mean_remove(x, L.N, L.d_part, s);
}

}  // namespace cav
