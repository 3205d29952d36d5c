// Internal data structures of the CAV-multigrid solver library.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/cavmg.h"

namespace cav {

// Host CSR over the 2 N^2 velocity unknowns of one level.
struct HostCSR {
  int64_t n = 0;                 // rows
  std::vector<int64_t> rowptr;   // n + 1
  std::vector<int32_t> col;
  std::vector<double> val;
  int64_t nnz() const { return rowptr.empty() ? 0 : rowptr.back(); }
};

// One explicit patch as the device kernels see it.
struct PatchRec {
  int32_t n;        // unknowns in the patch
  int32_t id;       // explicit patch index within its level
  int64_t slot;     // offset into slot_dof / delta
  int64_t fac;      // element offset into the factor arena of its precision
};

// An explicit patch in a multiplicative phase: precision picks the arena.
struct MultRec {
  int32_t n;
  int32_t f32;      // 1: factor in the FP32 arena
  int64_t slot;
  int64_t fac;
};

// Stencil coefficients of one level's rediscretised Stokes part.
struct StencilCoef {
  int N;
  double diag;   // rho/dt + 4 mu/h^2
  double off;    // mu/h^2 (A0 off-diagonal is -off)
  double invh;   // 1/h
};

struct Level {
  int N = 0;
  double h = 0;
  StencilCoef sc{};
  // E_E (unscaled), host copy with full row pointer; structural pattern kept
  HostCSR ee;
  // device: compressed rows of -dt * E_E for the operator apply
  int32_t n_erows = 0;
  int32_t* d_erow_id = nullptr;   // velocity unknown of each compressed row
  int32_t* d_erow_ptr = nullptr;  // n_erows + 1
  int32_t* d_ecol = nullptr;
  double* d_eval = nullptr;       // -dt * E_E
  // device: full row pointer (2N^2+1) into the same col/val arrays, for patch assembly
  int32_t* d_erow_full = nullptr;

  // patches (levels >= 1)
  bool has_patches = false;
  std::vector<uint8_t> cellflag;           // bit0 explicit seed, bit1 covered
  std::vector<int64_t> patch_off;          // all patches (N^2 + 1), for export
  std::vector<int32_t> patch_dofs;
  std::vector<int32_t> exp_cells;          // explicit patch -> seed cell
  std::vector<int64_t> exp_off;            // explicit patch -> slot offset (n_exp + 1)
  std::vector<int32_t> slot_dof_h;
  uint8_t* d_cellflag = nullptr;
  int32_t n_exp = 0;
  int64_t n_slots = 0;
  int32_t* d_slot_dof = nullptr;
  double* d_delta = nullptr;
  int32_t n_touched = 0;
  std::vector<int32_t> t_dof_h, t_ptr_h, t_slot_h;
  std::vector<double> t_inv_h;
  int32_t* d_t_dof = nullptr;
  double* d_t_inv = nullptr;
  int32_t* d_t_ptr = nullptr;
  int32_t* d_t_slot = nullptr;
  cav_level_stats stats{};
  // multiplicative sweep: explicit patches in colour phases
  std::vector<int32_t> ph_ptr;            // n_phases + 1 offsets into ph_exp
  std::vector<int32_t> ph_exp;            // explicit patch ids, phase-major
  MultRec* d_mrec = nullptr;              // records in ph_exp order
  int32_t mrec_max_n = 0;
  std::vector<double> ph_bytes;           // algorithmic bytes of each phase launch
  size_t mx_lds = 0;                      // dynamic LDS of the phase kernel

  // factors
  bool factored = false;
  double* d_std_inv = nullptr;            // 25 doubles, role order (u_l, u_r, v_b, v_t, p)
  std::vector<PatchRec> rec64_h, rec32_h; // sorted by n descending
  PatchRec* d_rec64 = nullptr;
  PatchRec* d_rec32 = nullptr;
  double* d_f64 = nullptr;
  float* d_f32 = nullptr;
  double bytes64 = 0, bytes32 = 0;        // algorithmic bytes of one GEMV launch per precision

  // per-level vectors (3 N^2)
  double *d_b = nullptr, *d_x = nullptr, *d_r = nullptr, *d_z = nullptr;
  double* d_part = nullptr;               // reduction partials
};

struct Ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  std::string err;
  int n_levels = 0;
  double rho = 1, mu = 0.01, dt = 1e-3;
  std::vector<Level> lv;                  // 0 = coarsest
  bool built = false, patched = false, factored = false;
  int family = CAV_FAMILY_CAV;
  double alpha = 0.7;
  int pre = 1, post = 1;
  int smoother = CAV_SMOOTHER_ADDITIVE;
  // coarsest bordered inverse (nb x nb, column-major) and its column permutation
  int nc = 0;                              // bordered size
  double* d_cinv = nullptr;
  int32_t* d_cperm = nullptr;
  // FGMRES workspace
  int ws_maxit = 0;
  int64_t ws_n = 0;  // vector length the workspace was sized for
  double *d_V = nullptr, *d_Z = nullptr, *d_w = nullptr, *d_bb = nullptr;
  double *d_h = nullptr, *d_part = nullptr;
  double* h_pinned = nullptr;
  std::vector<void*> allocs;
  // live timing of the explicit-patch GEMV and of whole V-cycles (HIP events)
  bool timing = false;
  std::vector<hipEvent_t> ev_pool;
  size_t ev_used = 0;
  std::vector<std::pair<int, double>> kt_marks;   // (event index of the start, bytes)
  std::vector<std::pair<int, int>> vc_marks;      // event indices around each V-cycle
};

hipEvent_t next_event(Ctx& c);
inline void timing_begin(Ctx& c, hipStream_t s) {
  if (!c.timing) return;
  hipEvent_t e = next_event(c);
  c.kt_marks.push_back({int(c.ev_used - 1), 0.0});
  (void)hipEventRecord(e, s);
}
inline void timing_end(Ctx& c, hipStream_t s, double bytes) {
  if (!c.timing) return;
  hipEvent_t e = next_event(c);
  c.kt_marks.back().second = bytes;
  (void)hipEventRecord(e, s);
}

// ---- host setup (setup_host.cpp) ----
struct Structure {
  int M = 0;
  std::vector<double> X, omega;
  HostCSR E;  // 2M x 2M, component interleaved
};
cav_status make_structure(const cav_structure_desc* st, Structure& out, std::string& err);
void assemble_ee_finest(int N, const Structure& s, HostCSR& ee);
void galerkin_coarsen(int Nc, const HostCSR& fine, HostCSR& coarse);
void build_patches(int N, const HostCSR& ee, int family, Level& L);

// ---- device launches (kernels_*.hip) ----
void launch_apply_op(const Level& L, const double* x, double* y, const double* b, hipStream_t s);
void launch_restrict(const Level& Lf, const double* rf, double* bc, hipStream_t s);
void launch_prolong_add(const Level& Lf, const double* xc, double* xf, hipStream_t s);
void launch_smoother(Ctx& c, Level& L, const double* b, double* x, bool zero_guess, hipStream_t s);
void launch_mult_smoother(Ctx& c, Level& L, const double* b, double* x, bool zero_guess, hipStream_t s);
void launch_fill(double* x, double v, int64_t n, hipStream_t s);
void colour_explicit(int N, const HostCSR& ee, Level& L);
void launch_coarse_solve(const Ctx& c, const double* b, double* x, hipStream_t s);
cav_status factor_level(Ctx& c, Level& L, int precision, double cond_threshold, cav_factor_stats* st);
cav_status factor_coarse(Ctx& c);

// vector helpers (kernels_grid.hip)
void launch_dots(const double* V, int64_t ldv, int k, const double* w, int64_t n, double* part, int nblk,
                 double* out, hipStream_t s);
void launch_multi_axpy(double* w, const double* V, int64_t ldv, int k, const double* coef, double sign, int64_t n,
                       hipStream_t s);
void launch_scale(double* y, const double* x, const double* denom, int64_t n, hipStream_t s);
void launch_pressure_mean_remove(double* x, int N, double* part, hipStream_t s);
void launch_block_sum(const double* x, int64_t n, double* part, double* out, hipStream_t s);
int dots_blocks(int64_t n);

void* dev_alloc(Ctx& c, size_t bytes);
void dev_free(Ctx& c, void* p);

}  // namespace cav

#define CAV_HIP(call)                                                                 \
  do {                                                                                \
    hipError_t e_ = (call);                                                           \
    if (e_ != hipSuccess) throw cav::HipError(std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

namespace cav {
struct HipError {
  std::string msg;
  explicit HipError(std::string m) : msg(std::move(m)) {}
};
struct StatusError {
  cav_status st;
  std::string msg;
  StatusError(cav_status s, std::string m) : st(s), msg(std::move(m)) {}
};
}  // namespace cav
