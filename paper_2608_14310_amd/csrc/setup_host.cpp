// Host-side setup: force laws, interpolation weights, E_E = S E J on the finest
// level, Galerkin coarsening, and patch construction (Sections 2-4).
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstring>
#include <map>
#include <thread>

#include "cav_internal.hpp"

namespace cav {

namespace {

inline int pmod(int64_t a, int n) {
  int64_t r = a % n;
  return int(r < 0 ? r + n : r);
}

// f(state, i) for every i in [0, n) on up to 16 host threads, items handed out
// in grains from a shared counter (the work per item is very uneven: patches
// near the structure are large). make_state() builds each thread's scratch
// once. Every item writes only its own output, so the result does not depend
// on the schedule.
template <typename MS, typename F>
void parallel_items(int64_t n, int64_t grain, MS&& make_state, F&& f) {
  int nt = int(std::min<unsigned>(std::max(1u, std::thread::hardware_concurrency()), 16u));
  if (n <= grain) nt = 1;
  std::atomic<int64_t> next{0};
  auto work = [&] {
    auto st = make_state();
    for (;;) {
      const int64_t b = next.fetch_add(grain);
      if (b >= n) break;
      const int64_t e = std::min(n, b + grain);
      for (int64_t i = b; i < e; ++i) f(st, i);
    }
  };
  if (nt <= 1) {
    work();
    return;
  }
  std::vector<std::thread> th;
  for (int t = 0; t < nt; ++t) th.emplace_back(work);
  for (auto& x : th) x.join();
}

// Rows [0, nrows) of a sparse matrix with ncols columns, built in parallel
// blocks of rows: row(f, add) calls add(g, v) for every contribution to row f
// in a fixed order; the contributions to one column are summed in that order
// and the row is stored with ascending columns. skip(f0, f1) may report a
// block of rows without any contribution. The blocks are concatenated in
// order, so the result does not depend on the schedule.
template <typename Skip, typename Row>
void build_rows(int64_t nrows, int64_t ncols, HostCSR& out, Skip&& skip, Row&& row) {
  constexpr int64_t RB = 1024;
  const int64_t nblk = (nrows + RB - 1) / RB;
  struct Block {
    std::vector<int32_t> col;
    std::vector<double> val;
    std::vector<int64_t> len;
  };
  struct Acc {
    std::vector<double> acc;
    std::vector<int64_t> mark;
    std::vector<int32_t> touched;
  };
  std::vector<Block> blocks(nblk);
  parallel_items(
      nblk, 1, [] { return Acc{}; },
      [&](Acc& A, int64_t b) {
        Block& B = blocks[b];
        const int64_t f0 = b * RB, f1 = std::min(nrows, f0 + RB);
        B.len.assign(f1 - f0, 0);
        if (skip(f0, f1)) return;
        if (A.acc.empty()) {
          A.acc.assign(ncols, 0.0);
          A.mark.assign(ncols, -1);
        }
        for (int64_t f = f0; f < f1; ++f) {
          A.touched.clear();
          row(f, [&](int32_t g, double v) {
            if (A.mark[g] != f) {
              A.mark[g] = f;
              A.acc[g] = 0.0;
              A.touched.push_back(g);
            }
            A.acc[g] += v;
          });
          std::sort(A.touched.begin(), A.touched.end());
          for (int32_t g : A.touched) {
            B.col.push_back(g);
            B.val.push_back(A.acc[g]);
          }
          B.len[f - f0] = int64_t(A.touched.size());
        }
      });
  out.n = nrows;
  out.rowptr.assign(nrows + 1, 0);
  int64_t total = 0;
  for (const Block& B : blocks) total += int64_t(B.col.size());
  out.col.clear();
  out.val.clear();
  out.col.reserve(size_t(total));
  out.val.reserve(size_t(total));
  for (int64_t b = 0; b < nblk; ++b) {
    const Block& B = blocks[b];
    const int64_t f0 = b * RB;
    for (size_t k = 0; k < B.len.size(); ++k) out.rowptr[f0 + int64_t(k) + 1] = out.rowptr[f0 + int64_t(k)] + B.len[k];
    out.col.insert(out.col.end(), B.col.begin(), B.col.end());
    out.val.insert(out.val.end(), B.val.begin(), B.val.end());
  }
}

// Peskin's four-point kernel (the textbook closed form used in Section 2).
inline double phi4(double r) {
  double a = std::fabs(r);
  if (a <= 1.0) return (3.0 - 2.0 * a + std::sqrt(std::max(1.0 + 4.0 * a - 4.0 * a * a, 0.0))) * 0.125;
  if (a <= 2.0) return (5.0 - 2.0 * a - std::sqrt(std::max(-7.0 + 12.0 * a - 4.0 * a * a, 0.0))) * 0.125;
  return 0.0;
}

// Kernel support of marker k, component c on an N grid: 16 faces and weights.
// u faces sit at (i, j+1/2) h, v faces at (i+1/2, j) h; the 4x4 box starts at
// floor(X/h - sigma) - 1 on each axis and every face of the box is kept.
struct Support {
  int32_t face[16];
  double w[16];
};

inline void support(int N, double x, double y, int c, Support& s) {
  const double h = 1.0 / N;
  const double sx = (c == 0) ? 0.0 : 0.5, sy = (c == 0) ? 0.5 : 0.0;
  const double gx = x / h - sx, gy = y / h - sy;
  const int64_t i0 = int64_t(std::floor(gx)) - 1, j0 = int64_t(std::floor(gy)) - 1;
  double wx[4], wy[4];
  for (int a = 0; a < 4; ++a) {
    wx[a] = phi4(double(i0 + a) - gx);
    wy[a] = phi4(double(j0 + a) - gy);
  }
  const int64_t base = int64_t(c) * N * N;
  for (int a = 0; a < 4; ++a)
    for (int b = 0; b < 4; ++b) {
      s.face[a * 4 + b] = int32_t(base + int64_t(pmod(i0 + a, N)) * N + pmod(j0 + b, N));
      s.w[a * 4 + b] = wx[a] * wy[b];
    }
}

// Scalar elasticity of one segment, as (row, col, val) triplets in marker indices.
void segment_law(int law, double kt, double ks, double kb, int m0, int M, bool closed, double ds,
                 std::map<std::pair<int, int>, double>& acc) {
  auto add = [&](int a, int b, double v) { acc[{m0 + a, m0 + b}] += v; };
  auto wrap = [&](int k) { return ((k % M) + M) % M; };
  if (law == CAV_LAW_TARGET) {
    for (int k = 0; k < M; ++k) add(k, k, -kt);
  } else if (law == CAV_LAW_MEMBRANE) {
    const double c = ks / (ds * ds);
    for (int k = 0; k < M; ++k) {
      add(k, wrap(k - 1), c);
      add(k, k, -2.0 * c);
      add(k, wrap(k + 1), c);
    }
  } else if (law == CAV_LAW_BEAM_CLOSED) {
    const double c = -kb / (ds * ds * ds * ds);
    const double st[5] = {1, -4, 6, -4, 1};
    for (int k = 0; k < M; ++k)
      for (int o = -2; o <= 2; ++o) add(k, wrap(k + o), c * st[o + 2]);
  } else if (law == CAV_LAW_BEAM_OPEN) {
    const double cb = -kb / (ds * ds * ds * ds), cs = -ks / (ds * ds);
    const double d2[3] = {1, -2, 1};
    for (int r = 0; r + 2 < M; ++r)               // -(kb/ds^4) D2^T D2
      for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) add(r + a, r + b, cb * d2[a] * d2[b]);
    const double d1[2] = {-1, 1};
    for (int r = 0; r + 1 < M; ++r)               // -(ks/ds^2) D1^T D1
      for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b) add(r + a, r + b, cs * d1[a] * d1[b]);
  }
}

}  // namespace

// Tangent of the clamped flexible fibre's force (Section 5.3). The force is
// F = -(1/ds) grad(U) for the total energy U of the bending, stretching,
// position and tangent terms, so E = -(1/ds) Hess(U). Each term's Hessian is
// formed from its own variables (link vectors, or the clamp coordinates) and
// scattered onto the markers it involves; the stored pattern is every 2 x 2
// block of markers at most two apart.
namespace {
// The configuration at which the fibre energies are evaluated: positions Xe
// (2M) and links D (2(M-1)). With a displacement the links are updated
// incrementally (Section 5.3), D_k = D_k^0 + (disp_{k+1} - disp_k), where D^0
// is the caller's carried links or else X_{k+1} - X_k: on a nearly straight
// fibre the cross products of the bending term are far below the positions'
// rounding, so differences of absolute positions would lose them.
cav_status fibre_configuration(const cav_structure_desc* st, int M, std::vector<double>& Xe,
                               std::vector<double>& D, std::string& err) {
  const size_t nx = 2 * size_t(M), nd = 2 * size_t(M - 1);
  auto finite = [&](const double* a, size_t n, const char* what) {
    for (size_t k = 0; k < n; ++k)
      if (!std::isfinite(a[k])) { err = what; return false; }
    return true;
  };
  if (st->X_force && !finite(st->X_force, nx, "non-finite X_force")) return CAV_ERR_INVALID_ARG;
  if (st->X_disp && !finite(st->X_disp, nx, "non-finite X_disp")) return CAV_ERR_INVALID_ARG;
  if (st->links && !finite(st->links, nd, "non-finite links")) return CAV_ERR_INVALID_ARG;
  const double* X0 = (st->X_force && !st->X_disp) ? st->X_force : st->X;
  Xe.assign(X0, X0 + nx);
  D.resize(nd);
  for (int k = 0; k + 1 < M; ++k)
    for (int c = 0; c < 2; ++c)
      D[2 * k + c] = (st->links && X0 == st->X) ? st->links[2 * k + c] : X0[2 * (k + 1) + c] - X0[2 * k + c];
  if (st->X_disp) {
    const double* u = st->X_disp;
    for (size_t k = 0; k < nx; ++k) Xe[k] += u[k];
    for (int k = 0; k + 1 < M; ++k)
      for (int c = 0; c < 2; ++c) D[2 * k + c] += u[2 * (k + 1) + c] - u[2 * k + c];
  }
  return CAV_OK;
}

cav_status fibre_law(const cav_structure_desc* st, Structure& s, std::string& err) {
  const int M = s.M;
  if (st->n_segments != 1 || !st->seg_start || !st->seg_closed || !st->seg_ds) {
    err = "fibre law needs exactly one segment"; return CAV_ERR_INVALID_ARG;
  }
  if (st->seg_start[0] != 0 || st->seg_start[1] != M) { err = "seg_start must run from 0 to M"; return CAV_ERR_INVALID_ARG; }
  if (st->seg_closed[0]) { err = "fibre law needs an open segment"; return CAV_ERR_INVALID_ARG; }
  if (M < 3) { err = "fibre law needs M >= 3"; return CAV_ERR_INVALID_ARG; }
  const int m = st->clamp_marker;
  if (m < 1 || m > M - 2) { err = "clamp_marker must lie in [1, M-2]"; return CAV_ERR_INVALID_ARG; }
  const double ds = st->seg_ds[0];
  if (!(ds > 0) || !std::isfinite(ds)) { err = "segment spacing must be positive"; return CAV_ERR_INVALID_ARG; }
  const double EI = st->kappa_b, Ks = st->kappa_s, Kp = st->K_p, Kt = st->K_t;
  for (double v : {EI, Ks, Kp, Kt, st->clamp_x, st->clamp_y})
    if (!std::isfinite(v)) { err = "non-finite fibre parameter"; return CAV_ERR_INVALID_ARG; }
  std::vector<double> Xe, D;
  if (const cav_status v = fibre_configuration(st, M, Xe, D, err); v != CAV_OK) return v;
  // band storage: B[i][d][a][b] = Hess(U) block (marker i, marker i+d-2), d in 0..4
  std::vector<double> B(size_t(M) * 5 * 4, 0.0);
  auto blk = [&](int i, int j, int a, int b) -> double& {
    return B[((size_t(i) * 5 + size_t(j - i + 2)) * 2 + a) * 2 + b];
  };
  auto link = [&](int k, int c) { return D[2 * k + c]; };
  // stretching: U_k = Ks/(2ds) (|d|-ds)^2 with d = X_{k+1} - X_k;
  // d2U_k/dd2 = (Ks/ds) [ (1 - ds/|d|) I + ds d d^T / |d|^3 ]
  for (int k = 0; k + 1 < M; ++k) {
    const double d[2] = {link(k, 0), link(k, 1)};
    const double len = std::hypot(d[0], d[1]);
    if (!(len > 0)) { err = "coincident fibre markers"; return CAV_ERR_INVALID_ARG; }
    for (int a = 0; a < 2; ++a)
      for (int b = 0; b < 2; ++b) {
        const double A = Ks / ds * ((a == b ? 1.0 - ds / len : 0.0) + ds * d[a] * d[b] / (len * len * len));
        blk(k, k, a, b) += A;
        blk(k + 1, k + 1, a, b) += A;
        blk(k, k + 1, a, b) -= A;
        blk(k + 1, k, a, b) -= A;
      }
  }
  // bending: U_k = EI/(2ds^5) c^2, c = p0 q1 - p1 q0 with p = D_k, q = D_{k+1};
  // in the variables v = (p0, p1, q0, q1): grad c = (q1, -q0, -p1, p0) and
  // Hess c has +1 at (p0, q1), -1 at (p1, q0) and their transposes.
  // Marker k+r moves p by sp[r] and q by sq[r].
  static const double sp[3] = {-1.0, 1.0, 0.0}, sq[3] = {0.0, -1.0, 1.0};
  const double wb = EI / std::pow(ds, 5);
  for (int k = 0; k + 2 < M; ++k) {
    const double p0 = link(k, 0), p1 = link(k, 1), q0 = link(k + 1, 0), q1 = link(k + 1, 1);
    const double c = p0 * q1 - p1 * q0;
    const double g[4] = {q1, -q0, -p1, p0};
    double Hv[4][4];
    for (int u = 0; u < 4; ++u)
      for (int v = 0; v < 4; ++v) Hv[u][v] = wb * g[u] * g[v];
    Hv[0][3] += wb * c; Hv[3][0] += wb * c;
    Hv[1][2] -= wb * c; Hv[2][1] -= wb * c;
    for (int r = 0; r < 3; ++r)
      for (int t = 0; t < 3; ++t)
        for (int a = 0; a < 2; ++a)
          for (int b = 0; b < 2; ++b)
            blk(k + r, k + t, a, b) += sp[r] * sp[t] * Hv[a][b] + sp[r] * sq[t] * Hv[a][2 + b] +
                                       sq[r] * sp[t] * Hv[2 + a][b] + sq[r] * sq[t] * Hv[2 + a][2 + b];
  }
  // position penalty on marker m; tangent penalty on the central difference
  // g = (X_{m+1} - X_{m-1})/(2ds): d2/dX2 of Kt/2 |g - e_x|^2 = Kt/(4ds^2) [[I, -I], [-I, I]]
  const double wt = Kt / (4.0 * ds * ds);
  for (int a = 0; a < 2; ++a) {
    blk(m, m, a, a) += Kp;
    blk(m - 1, m - 1, a, a) += wt;
    blk(m + 1, m + 1, a, a) += wt;
    blk(m - 1, m + 1, a, a) -= wt;
    blk(m + 1, m - 1, a, a) -= wt;
  }
  HostCSR& E = s.E;
  E.rowptr.assign(E.n + 1, 0);
  E.col.clear();
  E.val.clear();
  for (int i = 0; i < M; ++i)
    for (int a = 0; a < 2; ++a) {
      for (int j = std::max(0, i - 2); j <= std::min(M - 1, i + 2); ++j)
        for (int b = 0; b < 2; ++b) {
          const double v = -blk(i, j, a, b) / ds;
          if (!std::isfinite(v)) { err = "non-finite E value"; return CAV_ERR_INVALID_ARG; }
          E.col.push_back(2 * j + b);
          E.val.push_back(v);
        }
      E.rowptr[2 * int64_t(i) + a + 1] = int64_t(E.col.size());
    }
  return CAV_OK;
}
}  // namespace

// Force density of the clamped fibre, F = -(1/ds) grad(U) (Section 5.3), at
// the configuration fibre_configuration forms: each term's gradient in its own
// variables (links, clamp coordinates), scattered onto the markers it involves.
cav_status fibre_force(const cav_structure_desc* st, std::vector<double>& F, std::string& err) {
  Structure s;
  const cav_status v = make_structure(st, s, err);  // validates the descriptor and the parameters
  if (v != CAV_OK) return v;
  if (st->law != CAV_LAW_FIBRE) { err = "a force is defined here for the fibre law only"; return CAV_ERR_INVALID_ARG; }
  const int M = s.M, m = st->clamp_marker;
  const double ds = st->seg_ds[0];
  const double EI = st->kappa_b, Ks = st->kappa_s, Kp = st->K_p, Kt = st->K_t;
  std::vector<double> X, D;
  if (const cav_status c = fibre_configuration(st, M, X, D, err); c != CAV_OK) return c;
  auto link = [&](int k, int c) { return D[2 * k + c]; };
  std::vector<double> G(2 * size_t(M), 0.0);  // grad(U)
  // stretching: dU_k/dd = Ks/ds (|d| - ds) d/|d|, d = X_{k+1} - X_k
  for (int k = 0; k + 1 < M; ++k) {
    const double d0 = link(k, 0), d1 = link(k, 1);
    const double len = std::hypot(d0, d1);
    const double f = Ks / ds * (len - ds) / len;
    G[2 * k] -= f * d0;
    G[2 * k + 1] -= f * d1;
    G[2 * (k + 1)] += f * d0;
    G[2 * (k + 1) + 1] += f * d1;
  }
  // bending: dU_k/dv = EI/ds^5 c grad(c), v = (p, q) = (D_k, D_{k+1})
  const double wb = EI / std::pow(ds, 5);
  for (int k = 0; k + 2 < M; ++k) {
    const double p0 = link(k, 0), p1 = link(k, 1), q0 = link(k + 1, 0), q1 = link(k + 1, 1);
    const double c = wb * (p0 * q1 - p1 * q0);
    const double gp0 = c * q1, gp1 = -c * q0, gq0 = -c * p1, gq1 = c * p0;
    G[2 * k] -= gp0;
    G[2 * k + 1] -= gp1;
    G[2 * (k + 1)] += gp0 - gq0;
    G[2 * (k + 1) + 1] += gp1 - gq1;
    G[2 * (k + 2)] += gq0;
    G[2 * (k + 2) + 1] += gq1;
  }
  // clamp: position penalty on marker m, tangent penalty on the central
  // difference X_{m+1} - X_{m-1} = D_{m-1} + D_m
  G[2 * m] += Kp * (X[2 * m] - st->clamp_x);
  G[2 * m + 1] += Kp * (X[2 * m + 1] - st->clamp_y);
  const double t0 = (link(m - 1, 0) + link(m, 0)) / (2.0 * ds) - 1.0;
  const double t1 = (link(m - 1, 1) + link(m, 1)) / (2.0 * ds);
  const double wt = Kt / (2.0 * ds);
  G[2 * (m + 1)] += wt * t0;
  G[2 * (m + 1) + 1] += wt * t1;
  G[2 * (m - 1)] -= wt * t0;
  G[2 * (m - 1) + 1] -= wt * t1;
  F.resize(G.size());
  for (size_t k = 0; k < G.size(); ++k) {
    F[k] = -G[k] / ds;
    if (!std::isfinite(F[k])) { err = "non-finite fibre force"; return CAV_ERR_INVALID_ARG; }
  }
  return CAV_OK;
}

// The 16 faces and four-point kernel weights of every Lagrangian row (marker
// k, component c at row 2k + c), at the structure's positions X.
void ib_supports(int N, const Structure& s, std::vector<int32_t>& face, std::vector<double>& w) {
  const int64_t nr = 2 * int64_t(s.M);
  face.resize(size_t(nr) * 16);
  w.resize(size_t(nr) * 16);
  Support sg;
  for (int64_t r = 0; r < nr; ++r) {
    support(N, s.X[2 * (r / 2)], s.X[2 * (r / 2) + 1], int(r % 2), sg);
    for (int t = 0; t < 16; ++t) {
      face[size_t(r) * 16 + t] = sg.face[t];
      w[size_t(r) * 16 + t] = sg.w[t];
    }
  }
}

cav_status make_structure(const cav_structure_desc* st, Structure& s, std::string& err) {
  if (!st) { s.M = 0; s.E.n = 0; s.E.rowptr.assign(1, 0); return CAV_OK; }
  if (st->M < 0) { err = "M < 0"; return CAV_ERR_INVALID_ARG; }
  s.M = st->M;
  const int M = s.M;
  if (M > 0 && (!st->X || !st->omega)) { err = "X and omega are required when M > 0"; return CAV_ERR_INVALID_ARG; }
  s.X.assign(st->X, st->X + 2 * size_t(M));
  s.omega.assign(st->omega, st->omega + size_t(M));
  for (double v : s.X) if (!std::isfinite(v)) { err = "non-finite marker position"; return CAV_ERR_INVALID_ARG; }
  for (double v : s.omega) if (!std::isfinite(v)) { err = "non-finite quadrature weight"; return CAV_ERR_INVALID_ARG; }
  HostCSR& E = s.E;
  E.n = 2 * int64_t(M);
  if (st->law == CAV_LAW_CSR) {
    if (M > 0 && (!st->E_rowptr || !st->E_col || !st->E_val)) { err = "CSR law needs E arrays"; return CAV_ERR_INVALID_ARG; }
    E.rowptr.resize(E.n + 1);
    for (int64_t r = 0; r <= E.n; ++r) E.rowptr[r] = st->E_rowptr[r];
    if (E.rowptr[0] != 0 || E.rowptr[E.n] != st->E_nnz) { err = "E_rowptr inconsistent with E_nnz"; return CAV_ERR_INVALID_ARG; }
    for (int64_t r = 0; r < E.n; ++r)
      if (E.rowptr[r + 1] < E.rowptr[r]) { err = "E_rowptr not monotone"; return CAV_ERR_INVALID_ARG; }
    E.col.assign(st->E_col, st->E_col + st->E_nnz);
    E.val.assign(st->E_val, st->E_val + st->E_nnz);
    for (int64_t k = 0; k < st->E_nnz; ++k) {
      if (E.col[k] < 0 || E.col[k] >= E.n) { err = "E column out of range"; return CAV_ERR_INVALID_ARG; }
      if (!std::isfinite(E.val[k])) { err = "non-finite E value"; return CAV_ERR_INVALID_ARG; }
    }
    // structural symmetry
    std::vector<std::pair<int, int>> pairs, tr;
    for (int64_t r = 0; r < E.n; ++r)
      for (int64_t k = E.rowptr[r]; k < E.rowptr[r + 1]; ++k) {
        pairs.push_back({int(r), E.col[k]});
        tr.push_back({E.col[k], int(r)});
      }
    std::sort(pairs.begin(), pairs.end());
    std::sort(tr.begin(), tr.end());
    pairs.erase(std::unique(pairs.begin(), pairs.end()), pairs.end());
    tr.erase(std::unique(tr.begin(), tr.end()), tr.end());
    if (pairs != tr) { err = "E is not structurally symmetric"; return CAV_ERR_INVALID_ARG; }
    return CAV_OK;
  }
  if (st->law == CAV_LAW_FIBRE) return fibre_law(st, s, err);
  if (st->law < CAV_LAW_TARGET || st->law > CAV_LAW_BEAM_OPEN) { err = "unknown law"; return CAV_ERR_INVALID_ARG; }
  if (M > 0 && (st->n_segments < 1 || !st->seg_start || !st->seg_closed || !st->seg_ds)) {
    err = "segments are required for the built-in laws"; return CAV_ERR_INVALID_ARG;
  }
  std::map<std::pair<int, int>, double> acc;
  if (M > 0) {
    if (st->seg_start[0] != 0 || st->seg_start[st->n_segments] != M) { err = "seg_start must run from 0 to M"; return CAV_ERR_INVALID_ARG; }
    for (int g = 0; g < st->n_segments; ++g) {
      const int m0 = st->seg_start[g], m1 = st->seg_start[g + 1];
      if (m1 <= m0) { err = "empty segment"; return CAV_ERR_INVALID_ARG; }
      const bool closed = st->seg_closed[g] != 0;
      const double ds = st->seg_ds[g];
      if (!(ds > 0) || !std::isfinite(ds)) { err = "segment spacing must be positive"; return CAV_ERR_INVALID_ARG; }
      if ((st->law == CAV_LAW_MEMBRANE || st->law == CAV_LAW_BEAM_CLOSED) && !closed) {
        err = "membrane and closed-beam laws need closed segments"; return CAV_ERR_INVALID_ARG;
      }
      if (st->law == CAV_LAW_BEAM_OPEN && closed) { err = "open-beam law needs open segments"; return CAV_ERR_INVALID_ARG; }
      segment_law(st->law, st->kappa_t, st->kappa_s, st->kappa_b, m0, m1 - m0, closed, ds, acc);
    }
  }
  // interleave the scalar law onto both components
  std::vector<std::vector<std::pair<int, double>>> rows(M);
  for (auto& kv : acc) rows[kv.first.first].push_back({kv.first.second, kv.second});
  E.rowptr.assign(E.n + 1, 0);
  for (int k = 0; k < M; ++k)
    for (int c = 0; c < 2; ++c) {
      const int64_t r = 2 * int64_t(k) + c;
      for (auto& e : rows[k]) {
        E.col.push_back(2 * e.first + c);
        E.val.push_back(e.second);
      }
      E.rowptr[r + 1] = int64_t(E.col.size());
    }
  for (double v : E.val) if (!std::isfinite(v)) { err = "non-finite E value"; return CAV_ERR_INVALID_ARG; }
  return CAV_OK;
}

// E_E = (1/h^2) J^T (W E) J with W = diag(omega) on both components, accumulated
// row by row with a dense sparse accumulator. Every generated (row, col) pair
// is kept (structural pattern).
void assemble_ee_finest(int N, const Structure& s, HostCSR& ee) {
  const int64_t nv = 2 * int64_t(N) * N;
  const double h = 1.0 / N, ih2 = 1.0 / (h * h);
  const int64_t nr = 2 * int64_t(s.M);
  std::vector<Support> sup(nr);
  for (int64_t r = 0; r < nr; ++r) support(N, s.X[2 * (r / 2)], s.X[2 * (r / 2) + 1], int(r % 2), sup[r]);
  // face -> (Lagrangian row, weight), grouped by face with a counting sort
  std::vector<int64_t> fptr(nv + 1, 0);
  for (int64_t r = 0; r < nr; ++r)
    for (int t = 0; t < 16; ++t) fptr[sup[r].face[t] + 1]++;
  for (int64_t f = 0; f < nv; ++f) fptr[f + 1] += fptr[f];
  std::vector<int64_t> fr(fptr.back());
  std::vector<double> fw(fptr.back());
  {
    std::vector<int64_t> pos(fptr.begin(), fptr.end() - 1);
    for (int64_t r = 0; r < nr; ++r)
      for (int t = 0; t < 16; ++t) {
        const int64_t q = pos[sup[r].face[t]]++;
        fr[q] = r;
        fw[q] = sup[r].w[t];
      }
  }
  build_rows(
      nv, nv, ee, [&](int64_t f0, int64_t f1) { return fptr[f1] == fptr[f0]; },
      [&](int64_t f, auto&& add) {
        for (int64_t q = fptr[f]; q < fptr[f + 1]; ++q) {
          const int64_t r = fr[q];
          const double wf = fw[q] * s.omega[r / 2] * ih2;
          for (int64_t k = s.E.rowptr[r]; k < s.E.rowptr[r + 1]; ++k) {
            const double cf = wf * s.E.val[k];
            const Support& sg = sup[s.E.col[k]];
            for (int t = 0; t < 16; ++t) add(sg.face[t], cf * sg.w[t]);
          }
        }
      });
}

namespace {
// RT0 velocity prolongation stencils between a coarse grid Nc and fine grid 2Nc.
// pcol: coarse unknown -> (fine unknown, weight); prow: fine -> (coarse, weight).
inline int pcol(int Nc, int64_t F, int32_t* f, double* w) {
  const int Nf = 2 * Nc;
  const int64_t nc2 = int64_t(Nc) * Nc, nf2 = int64_t(Nf) * Nf;
  if (F < nc2) {
    const int I = int(F / Nc), J = int(F % Nc);
    int k = 0;
    for (int dj = 0; dj < 2; ++dj) {
      f[k] = int32_t(int64_t(pmod(2 * I, Nf)) * Nf + pmod(2 * J + dj, Nf)); w[k++] = 1.0;
      f[k] = int32_t(int64_t(pmod(2 * I + 1, Nf)) * Nf + pmod(2 * J + dj, Nf)); w[k++] = 0.5;
      f[k] = int32_t(int64_t(pmod(2 * I - 1, Nf)) * Nf + pmod(2 * J + dj, Nf)); w[k++] = 0.5;
    }
    return k;
  }
  const int64_t G = F - nc2;
  const int I = int(G / Nc), J = int(G % Nc);
  int k = 0;
  for (int di = 0; di < 2; ++di) {
    f[k] = int32_t(nf2 + int64_t(pmod(2 * I + di, Nf)) * Nf + pmod(2 * J, Nf)); w[k++] = 1.0;
    f[k] = int32_t(nf2 + int64_t(pmod(2 * I + di, Nf)) * Nf + pmod(2 * J + 1, Nf)); w[k++] = 0.5;
    f[k] = int32_t(nf2 + int64_t(pmod(2 * I + di, Nf)) * Nf + pmod(2 * J - 1, Nf)); w[k++] = 0.5;
  }
  return k;
}

inline int prow(int Nc, int64_t g, int32_t* G, double* w) {
  const int Nf = 2 * Nc;
  const int64_t nc2 = int64_t(Nc) * Nc, nf2 = int64_t(Nf) * Nf;
  if (g < nf2) {
    const int i = int(g / Nf), j = int(g % Nf);
    if (i % 2 == 0) { G[0] = int32_t(int64_t(i / 2) * Nc + j / 2); w[0] = 1.0; return 1; }
    G[0] = int32_t(int64_t((i - 1) / 2) * Nc + j / 2); w[0] = 0.5;
    G[1] = int32_t(int64_t(pmod((i + 1) / 2, Nc)) * Nc + j / 2); w[1] = 0.5;
    return 2;
  }
  const int64_t q = g - nf2;
  const int i = int(q / Nf), j = int(q % Nf);
  if (j % 2 == 0) { G[0] = int32_t(nc2 + int64_t(i / 2) * Nc + j / 2); w[0] = 1.0; return 1; }
  G[0] = int32_t(nc2 + int64_t(i / 2) * Nc + (j - 1) / 2); w[0] = 0.5;
  G[1] = int32_t(nc2 + int64_t(i / 2) * Nc + pmod((j + 1) / 2, Nc)); w[1] = 0.5;
  return 2;
}
}  // namespace

// E_E^(l-1) = R E_E^(l) P with R = P^T / 4, row by row (Section 4).
void galerkin_coarsen(int Nc, const HostCSR& fine, HostCSR& coarse) {
  const int64_t nvc = 2 * int64_t(Nc) * Nc;
  build_rows(
      nvc, nvc, coarse, [](int64_t, int64_t) { return false; },
      [&](int64_t F, auto&& add) {
        int32_t f[6], G[2];
        double wf[6], wg[2];
        const int nf = pcol(Nc, F, f, wf);
        for (int a = 0; a < nf; ++a) {
          const int64_t r = f[a];
          for (int64_t k = fine.rowptr[r]; k < fine.rowptr[r + 1]; ++k) {
            const double e = 0.25 * wf[a] * fine.val[k];
            const int ng = prow(Nc, fine.col[k], G, wg);
            for (int b = 0; b < ng; ++b) add(G[b], e * wg[b]);
          }
        }
      });
}

// Unknowns one unknown d reaches through a structural entry of K_E (itself
// included): MAC stencil neighbours and its E_E row.
template <typename V>
void visit_unknown_reach(int N, const HostCSR& ee, int64_t d, V&& visit) {
  const int64_t n2 = int64_t(N) * N, nv = 2 * n2;
  visit(d);
  if (d < n2) {                      // u_ij: u neighbours, p_ij, p_{i-1,j}, E_E row
    const int i = int(d / N), j = int(d % N);
    visit(int64_t(pmod(i + 1, N)) * N + j);
    visit(int64_t(pmod(i - 1, N)) * N + j);
    visit(int64_t(i) * N + pmod(j + 1, N));
    visit(int64_t(i) * N + pmod(j - 1, N));
    visit(nv + d);
    visit(nv + int64_t(pmod(i - 1, N)) * N + j);
  } else if (d < nv) {               // v_ij: v neighbours, p_ij, p_{i,j-1}, E_E row
    const int64_t q = d - n2;
    const int i = int(q / N), j = int(q % N);
    visit(n2 + int64_t(pmod(i + 1, N)) * N + j);
    visit(n2 + int64_t(pmod(i - 1, N)) * N + j);
    visit(n2 + int64_t(i) * N + pmod(j + 1, N));
    visit(n2 + int64_t(i) * N + pmod(j - 1, N));
    visit(nv + q);
    visit(nv + int64_t(i) * N + pmod(j - 1, N));
  } else {                           // p_ij: the four faces of its cell
    const int64_t q = d - nv;
    const int i = int(q / N), j = int(q % N);
    visit(q);
    visit(int64_t(pmod(i + 1, N)) * N + j);
    visit(n2 + q);
    visit(n2 + int64_t(i) * N + pmod(j + 1, N));
  }
  if (d < nv)
    for (int64_t k = ee.rowptr[d]; k < ee.rowptr[d + 1]; ++k) visit(ee.col[k]);
}

// Phases of the multiplicative sweep for the explicit patches: greedy colouring
// of the conflict graph (two patches conflict when one holds an unknown that
// the other's unknowns reach through a structural entry of K_E, itself
// included), visiting patches by decreasing size then cell index and giving
// each the smallest colour free among its coloured neighbours. Patches of one
// colour share no unknown and no coupling, so they can be applied at once.
//
// Every explicit patch is the unknown set V(C_e) of a cell set C_e (V(c): the
// four faces and the pressure of cell c), so the conflict graph is formed on
// cells: RC(c) holds the cells c' with V(c') meeting the reach of V(c), and
// e, o conflict iff some c in C_e has some c' of C_o in RC(c). This is the
// same relation as on unknowns, with a fraction of the work.
void colour_explicit(int N, const HostCSR& ee, Level& L) {
  const int64_t n2 = int64_t(N) * N;
  const int ne = L.n_exp;
  L.coloured = true;
  L.ph_ptr.assign(1, 0);
  L.ph_exp.clear();
  if (ne == 0) return;
  // cell owners: cell -> explicit patches whose cell set holds it
  std::vector<int32_t> cptr(n2 + 1, 0);
  for (int32_t c : L.exp_cov) cptr[c + 1]++;
  for (int64_t c = 0; c < n2; ++c) cptr[c + 1] += cptr[c];
  std::vector<int32_t> cown(cptr.back());
  {
    std::vector<int32_t> pos(cptr.begin(), cptr.end() - 1);
    for (int e = 0; e < ne; ++e)
      for (int64_t s = L.exp_cov_off[e]; s < L.exp_cov_off[e + 1]; ++s) cown[pos[L.exp_cov[s]]++] = e;
  }
  // RC(c) for every covered cell (index into `covered`)
  std::vector<int32_t> covered, cidx(n2, -1);
  for (int64_t c = 0; c < n2; ++c)
    if (cptr[c + 1] > cptr[c]) {
      cidx[c] = int32_t(covered.size());
      covered.push_back(int32_t(c));
    }
  std::vector<std::vector<int32_t>> rc(covered.size());
  auto cells_of = [&](int64_t d, int32_t* out) {   // cells whose V holds unknown d
    const int64_t nv = 2 * n2;
    if (d < n2) {
      const int a = int(d / N), b = int(d % N);
      out[0] = int32_t(d);
      out[1] = int32_t(int64_t(pmod(a - 1, N)) * N + b);
      return 2;
    }
    if (d < nv) {
      const int64_t q = d - n2;
      const int a = int(q / N), b = int(q % N);
      out[0] = int32_t(q);
      out[1] = int32_t(int64_t(a) * N + pmod(b - 1, N));
      return 2;
    }
    out[0] = int32_t(d - nv);
    return 1;
  };
  parallel_items(
      int64_t(covered.size()), 16, [&] { return std::vector<int32_t>(n2, -1); },
      [&](std::vector<int32_t>& mark, int64_t k) {
        const int32_t c = covered[k];
        const int a = c / N, b = c % N;
        const int64_t V[5] = {c, int64_t(pmod(a + 1, N)) * N + b, n2 + c, n2 + int64_t(a) * N + pmod(b + 1, N),
                              2 * n2 + c};
        std::vector<int32_t>& out = rc[k];
        for (int64_t d : V)
          visit_unknown_reach(N, ee, d, [&](int64_t r) {
            int32_t cc[2];
            const int m = cells_of(r, cc);
            for (int t = 0; t < m; ++t)
              if (mark[cc[t]] != c) {
                mark[cc[t]] = c;
                out.push_back(cc[t]);
              }
          });
      });
  std::vector<int> order(ne);
  for (int e = 0; e < ne; ++e) order[e] = e;
  auto np_of = [&](int e) { return L.exp_off[e + 1] - L.exp_off[e]; };
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
    if (np_of(a) != np_of(b)) return np_of(a) > np_of(b);
    return L.exp_cells[a] < L.exp_cells[b];
  });
  // conflict lists, independently per patch (in parallel); then the greedy pass
  std::vector<std::vector<int32_t>> nbr(ne);
  struct Marks {
    std::vector<int32_t> stamp, pmark;
  };
  parallel_items(
      ne, 8, [&] { return Marks{std::vector<int32_t>(n2, -1), std::vector<int32_t>(ne, -1)}; },
      [&](Marks& M, int64_t ee_) {
        const int e = int(ee_);
        std::vector<int32_t>& out = nbr[e];
        for (int64_t s = L.exp_cov_off[e]; s < L.exp_cov_off[e + 1]; ++s)
          for (int32_t c2 : rc[cidx[L.exp_cov[s]]]) {
            if (M.stamp[c2] == e) continue;
            M.stamp[c2] = e;
            for (int32_t q = cptr[c2]; q < cptr[c2 + 1]; ++q) {
              const int32_t o = cown[q];
              if (o != e && M.pmark[o] != e) {
                M.pmark[o] = e;
                out.push_back(o);
              }
            }
          }
      });
  std::vector<int> colour(ne, -1), cmark;
  int ncol = 0;
  for (int e : order) {
    cmark.resize(size_t(ncol) + 1, -1);
    for (int32_t q : nbr[e])
      if (colour[q] >= 0) cmark[colour[q]] = e;
    int c = 0;
    while (c < ncol && cmark[c] == e) ++c;
    colour[e] = c;
    if (c == ncol) ++ncol;
  }
  // phases: colour-major, explicit patches by ascending cell inside a colour
  std::vector<std::vector<int32_t>> by(ncol);
  for (int e = 0; e < ne; ++e) by[colour[e]].push_back(e);  // e ascends with the cell index
  for (int c = 0; c < ncol; ++c) {
    L.ph_exp.insert(L.ph_exp.end(), by[c].begin(), by[c].end());
    L.ph_ptr.push_back(int32_t(L.ph_exp.size()));
  }
  // predecessors of every patch in this order: its conflicting patches of an
  // earlier colour (the conflict relation is symmetric: the reach of an
  // unknown through the K_E pattern is, and the colouring relies on it)
  L.pred_ptr.assign(size_t(ne) + 1, 0);
  for (int e = 0; e < ne; ++e) {
    int64_t k = 0;
    for (int32_t q : nbr[e]) k += colour[q] < colour[e];
    L.pred_ptr[e + 1] = L.pred_ptr[e] + k;
  }
  L.pred.resize(size_t(L.pred_ptr[ne]));
  parallel_items(
      ne, 64, [] { return 0; },
      [&](int&, int64_t e) {
        int64_t o = L.pred_ptr[e];
        for (int32_t q : nbr[e])
          if (colour[q] < colour[e]) L.pred[o++] = q;
      });
}

// CAV patch family (Eq. cav_patch_set) on one level, plus the arrays the
// smoother needs: cell flags, explicit patch slots and the unknown -> slot
// transpose with 1/cnt weights (Appendix A's partition of unity).
// B(b,o) box family (Section 3.1): one patch per b x b block, the union of the
// Vanka patches of the block expanded by o cells on every side; restricted
// injection keeps the unknowns of the unexpanded block (Section 3.3). Every
// cell is flagged as handled by an explicit patch (no shared standard
// patches); the touched lists hold the injected slots only, with weight 1.
namespace {
// Bits 2, 3, 4 of a cell's flag: its u, v, p unknown is on the touched list
// (updated by the touched pass, not by the shared-inverse pass).
void mark_touched(int N, Level& L) {
  const int64_t n2 = int64_t(N) * N;
  for (uint8_t& f : L.cellflag) f &= 3;
  for (int32_t d : L.t_dof_h) L.cellflag[size_t(d % n2)] |= uint8_t(4 << (d / n2));
}
}  // namespace

void build_box_patches(int N, const HostCSR& ee, int b, int o, Level& L) {
  const int64_t n2 = int64_t(N) * N, n = 3 * n2;
  auto vanka = [&](int i, int j, int32_t* d) {
    d[0] = int32_t(int64_t(i) * N + j);
    d[1] = int32_t(int64_t(pmod(i + 1, N)) * N + j);
    d[2] = int32_t(n2 + int64_t(i) * N + j);
    d[3] = int32_t(n2 + int64_t(i) * N + pmod(j + 1, N));
    d[4] = int32_t(2 * n2 + int64_t(i) * N + j);
  };
  L.cellflag.assign(n2, 1);
  L.patch_off.assign(n2 + 1, 0);
  L.patch_dofs.clear();
  L.exp_cells.clear();
  L.exp_off.assign(1, 0);
  L.exp_cov_off.assign(1, 0);
  L.exp_cov.clear();
  L.slot_dof_h.clear();
  L.slot_mask_h.clear();
  std::vector<int32_t> mark(n, -1), core(n, -1), cmark(n2, -1);
  std::vector<int32_t> dofs;
  for (int i = 0; i < N; ++i)
    for (int j = 0; j < N; ++j) {
      const int32_t cell = int32_t(int64_t(i) * N + j);
      int64_t len = 0;
      if (i % b == 0 && j % b == 0) {
        dofs.clear();
        int32_t d[5];
        for (int r = -o; r < b + o; ++r)
          for (int t = -o; t < b + o; ++t) {
            vanka(pmod(i + r, N), pmod(j + t, N), d);
            if (cmark[d[4] - 2 * n2] != cell) {
              cmark[d[4] - 2 * n2] = cell;
              L.exp_cov.push_back(int32_t(d[4] - 2 * n2));
            }
            for (int k = 0; k < 5; ++k)
              if (mark[d[k]] != cell) {
                mark[d[k]] = cell;
                dofs.push_back(d[k]);
              }
          }
        for (int r = 0; r < b; ++r)
          for (int t = 0; t < b; ++t) {
            vanka(pmod(i + r, N), pmod(j + t, N), d);
            for (int k = 0; k < 5; ++k) core[d[k]] = cell;
          }
        std::sort(dofs.begin(), dofs.end());
        L.patch_dofs.insert(L.patch_dofs.end(), dofs.begin(), dofs.end());
        L.exp_cells.push_back(cell);
        L.exp_off.push_back(L.exp_off.back() + int64_t(dofs.size()));
        L.exp_cov_off.push_back(int64_t(L.exp_cov.size()));
        for (int32_t q : dofs) {
          L.slot_dof_h.push_back(q);
          L.slot_mask_h.push_back(core[q] == cell ? 1 : 0);
        }
        len = int64_t(dofs.size());
      }
      L.patch_off[cell + 1] = L.patch_off[cell] + len;
    }
  L.n_exp = int32_t(L.exp_cells.size());
  L.n_slots = int64_t(L.slot_dof_h.size());
  // unknown -> injected slots (ascending), weight 1
  std::vector<int32_t> nsl(n + 1, 0);
  for (int64_t sl = 0; sl < L.n_slots; ++sl)
    if (L.slot_mask_h[sl]) nsl[L.slot_dof_h[sl] + 1]++;
  L.t_dof_h.clear();
  L.t_ptr_h.assign(1, 0);
  std::vector<int64_t> start(n, -1);
  for (int64_t d = 0; d < n; ++d)
    if (nsl[d + 1] > 0) {
      start[d] = L.t_ptr_h.back();
      L.t_dof_h.push_back(int32_t(d));
      L.t_ptr_h.push_back(L.t_ptr_h.back() + nsl[d + 1]);
    }
  L.t_slot_h.assign(size_t(L.t_ptr_h.back()), 0);
  for (int64_t sl = 0; sl < L.n_slots; ++sl)
    if (L.slot_mask_h[sl]) L.t_slot_h[start[L.slot_dof_h[sl]]++] = int32_t(sl);
  L.t_inv_h.assign(L.t_dof_h.size(), 1.0);
  L.n_touched = int32_t(L.t_dof_h.size());
  mark_touched(N, L);
  colour_explicit(N, ee, L);
  cav_level_stats& st = L.stats;
  st.N = N;
  st.n_patches = L.n_exp;
  st.n_explicit = L.n_exp;
  st.max_np = 0;
  st.sum_np2 = 0;
  for (int32_t e = 0; e < L.n_exp; ++e) {
    const int64_t np = L.exp_off[e + 1] - L.exp_off[e];
    st.max_np = std::max<int32_t>(st.max_np, int32_t(np));
    st.sum_np2 += np * np;
  }
  st.avg_np = L.n_exp ? double(L.patch_dofs.size()) / double(L.n_exp) : 0.0;
  st.ee_nnz = ee.nnz();
  st.n_touched = L.n_touched;
}

void build_patch_sets(int N, const HostCSR& ee, int family, Level& L) {
  L.slot_mask_h.clear();
  const int64_t n2 = int64_t(N) * N, nv = 2 * n2, n = 3 * n2;
  auto U_of = [&](int i, int j, int32_t* U) {
    U[0] = int32_t(int64_t(i) * N + j);
    U[1] = int32_t(int64_t(pmod(i + 1, N)) * N + j);
    U[2] = int32_t(n2 + int64_t(i) * N + j);
    U[3] = int32_t(n2 + int64_t(i) * N + pmod(j + 1, N));
  };
  auto rowlen = [&](int64_t d) { return ee.rowptr[d + 1] - ee.rowptr[d]; };
  L.cellflag.assign(n2, 0);
  L.patch_off.assign(n2 + 1, 0);

  // rows of cells in parallel; each range keeps its own output, merged in order
  struct Part {
    std::vector<int32_t> dofs, plen, ecells, slot, elen, cov, clen;
  };
  std::vector<Part> parts(N);
  struct Scratch {
    std::vector<int32_t> cmark, dmark, cells, dofs, uhat;
  };
  parallel_items(
      N, 1, [&] { return Scratch{std::vector<int32_t>(n2, -1), std::vector<int32_t>(n, -1), {}, {}, {}}; },
      [&](Scratch& S, int64_t row) {
    std::vector<int32_t>& cmark = S.cmark;
    std::vector<int32_t>& dmark = S.dmark;
    std::vector<int32_t>& cells = S.cells;
    std::vector<int32_t>& dofs = S.dofs;
    Part& P = parts[row];
    const int i = int(row);
    for (int j = 0; j < N; ++j) {
      const int32_t cell = int32_t(int64_t(i) * N + j);
      int32_t U[4];
      U_of(i, j, U);
      bool anyrow = false;
      for (int k = 0; k < 4; ++k) anyrow |= rowlen(U[k]) > 0;
      dofs.clear();
      cells.clear();
      bool enlarged = false;
      if (anyrow && family == CAV_FAMILY_CAV) {
        // U_hat = U plus every velocity coupled to U through E_E (pattern is symmetric)
        std::vector<int32_t>& uhat = S.uhat;
        uhat.assign(U, U + 4);
        for (int k = 0; k < 4; ++k)
          for (int64_t q = ee.rowptr[U[k]]; q < ee.rowptr[U[k] + 1]; ++q) {
            const int32_t w = ee.col[q];
            if (w != U[0] && w != U[1] && w != U[2] && w != U[3]) { enlarged = true; uhat.push_back(w); }
          }
        if (enlarged) {
          for (int32_t w : uhat) {   // C(w): the two cells whose divergence rows hold w
            int32_t c2[2];
            if (w < n2) {
              const int a = w / N, b = w % N;
              c2[0] = int32_t(int64_t(pmod(a - 1, N)) * N + b);
              c2[1] = w;
            } else {
              const int32_t q = int32_t(w - n2);
              const int a = q / N, b = q % N;
              c2[0] = int32_t(int64_t(a) * N + pmod(b - 1, N));
              c2[1] = q;
            }
            for (int t = 0; t < 2; ++t)
              if (cmark[c2[t]] != cell) { cmark[c2[t]] = cell; cells.push_back(c2[t]); }
          }
          for (int32_t c : cells) {  // V(C): pressure and the four velocities of each cell
            int32_t Uc[4];
            U_of(c / N, c % N, Uc);
            const int32_t pc = int32_t(2 * n2 + c);
            for (int32_t d : {Uc[0], Uc[1], Uc[2], Uc[3], pc})
              if (dmark[d] != cell) { dmark[d] = cell; dofs.push_back(d); }
          }
        }
      }
      if (!enlarged) {
        dofs.assign(U, U + 4);
        dofs.push_back(int32_t(2 * n2 + cell));
        cells.assign(1, cell);
      }
      std::sort(dofs.begin(), dofs.end());
      P.dofs.insert(P.dofs.end(), dofs.begin(), dofs.end());
      P.plen.push_back(int32_t(dofs.size()));
      if (anyrow) {  // own factor whenever E_E enters the local matrix
        P.ecells.push_back(cell);
        P.slot.insert(P.slot.end(), dofs.begin(), dofs.end());
        P.elen.push_back(int32_t(dofs.size()));
        P.cov.insert(P.cov.end(), cells.begin(), cells.end());
        P.clen.push_back(int32_t(cells.size()));
      }
    }
  });
  // concatenate the rows' parts in row order: offsets by prefix sums, then
  // every row copies its part in parallel (each writes only its own ranges)
  {
    std::vector<int64_t> od(N + 1, 0), oe(N + 1, 0), os(N + 1, 0), oc(N + 1, 0);
    for (int r = 0; r < N; ++r) {
      const Part& P = parts[r];
      od[r + 1] = od[r] + int64_t(P.dofs.size());
      oe[r + 1] = oe[r] + int64_t(P.ecells.size());
      os[r + 1] = os[r] + int64_t(P.slot.size());
      oc[r + 1] = oc[r] + int64_t(P.cov.size());
    }
    L.patch_dofs.resize(size_t(od[N]));
    L.exp_cells.resize(size_t(oe[N]));
    L.exp_off.assign(size_t(oe[N]) + 1, 0);
    L.slot_dof_h.resize(size_t(os[N]));
    L.exp_cov.resize(size_t(oc[N]));
    L.exp_cov_off.assign(size_t(oe[N]) + 1, 0);
    parallel_items(
        N, 8, [] { return 0; },
        [&](int&, int64_t r) {
          const Part& P = parts[r];
          int64_t a = od[r];
          for (int j = 0; j < N; ++j) {
            a += P.plen[j];
            L.patch_off[r * N + j + 1] = a;
          }
          std::copy(P.dofs.begin(), P.dofs.end(), L.patch_dofs.begin() + od[r]);
          std::copy(P.slot.begin(), P.slot.end(), L.slot_dof_h.begin() + os[r]);
          std::copy(P.cov.begin(), P.cov.end(), L.exp_cov.begin() + oc[r]);
          int64_t sa = os[r], ca = oc[r];
          for (size_t k = 0; k < P.ecells.size(); ++k) {
            const int64_t e = oe[r] + int64_t(k);
            L.exp_cells[size_t(e)] = P.ecells[k];
            L.cellflag[P.ecells[k]] |= 1;   // a row's own cells
            sa += P.elen[k];
            ca += P.clen[k];
            L.exp_off[size_t(e) + 1] = sa;
            L.exp_cov_off[size_t(e) + 1] = ca;
          }
        });
    for (int32_t cc : L.exp_cov) L.cellflag[cc] |= 2;   // cells of other rows too: serial
  }
  L.n_exp = int32_t(L.exp_cells.size());
  L.n_slots = int64_t(L.slot_dof_h.size());
}

void build_patch_tables(int N, const HostCSR& ee, Level& L, bool colour) {
  const int64_t n2 = int64_t(N) * N, nv = 2 * n2, n = 3 * n2;
  // unknown -> slots transpose (counting sort, slots ascending within each unknown)
  std::vector<int32_t> nsl(n + 1, 0);
  for (int32_t d : L.slot_dof_h) nsl[d + 1]++;
  L.t_dof_h.clear();
  L.t_ptr_h.assign(1, 0);
  std::vector<int64_t> start(n, -1);
  for (int64_t d = 0; d < n; ++d)
    if (nsl[d + 1] > 0) {
      start[d] = L.t_ptr_h.back();
      L.t_dof_h.push_back(int32_t(d));
      L.t_ptr_h.push_back(L.t_ptr_h.back() + nsl[d + 1]);
    }
  L.t_slot_h.assign(L.n_slots, 0);
  for (int64_t sl = 0; sl < L.n_slots; ++sl) L.t_slot_h[start[L.slot_dof_h[sl]]++] = int32_t(sl);
  // cnt(d) = explicit patches holding d + shared standard patches holding d
  L.t_inv_h.resize(L.t_dof_h.size());
  for (size_t t = 0; t < L.t_dof_h.size(); ++t) {
    const int32_t d = L.t_dof_h[t];
    int cnt = L.t_ptr_h[t + 1] - L.t_ptr_h[t];
    int32_t inc[2];
    int ninc;
    if (d < n2) {
      const int a = d / N, b = d % N;
      inc[0] = int32_t(int64_t(pmod(a - 1, N)) * N + b); inc[1] = d; ninc = 2;
    } else if (d < nv) {
      const int32_t q = int32_t(d - n2);
      const int a = q / N, b = q % N;
      inc[0] = int32_t(int64_t(a) * N + pmod(b - 1, N)); inc[1] = q; ninc = 2;
    } else {
      inc[0] = int32_t(d - nv); ninc = 1;
    }
    for (int k = 0; k < ninc; ++k) cnt += (L.cellflag[inc[k]] & 1) ? 0 : 1;
    L.t_inv_h[t] = 1.0 / double(cnt);
  }
  L.n_touched = int32_t(L.t_dof_h.size());
  mark_touched(N, L);
  L.coloured = false;
  if (colour) colour_explicit(N, ee, L);

  // stats
  cav_level_stats& st = L.stats;
  st.N = N;
  st.n_patches = int32_t(n2);
  st.n_explicit = L.n_exp;
  st.max_np = 0;
  st.sum_np2 = 0;
  for (int64_t c = 0; c < n2; ++c) st.max_np = std::max<int32_t>(st.max_np, int32_t(L.patch_off[c + 1] - L.patch_off[c]));
  st.avg_np = double(L.patch_dofs.size()) / double(n2);
  for (int32_t e = 0; e < L.n_exp; ++e) {
    const int64_t np = L.exp_off[e + 1] - L.exp_off[e];
    st.sum_np2 += np * np;
  }
  st.ee_nnz = ee.nnz();
  st.n_touched = L.n_touched;
}

void build_patches(int N, const HostCSR& ee, int family, Level& L) {
  build_patch_sets(N, ee, family, L);
  build_patch_tables(N, ee, L);
}

}  // namespace cav
