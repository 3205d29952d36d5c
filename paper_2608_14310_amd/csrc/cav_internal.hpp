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

// Symmetric panel layout of one explicit patch inverse (n x n): panel k
// holds columns 16k .. 16k + w - 1 (w = min(16, n - 16k)) on rows 16k .. n - 1,
// column-major inside the panel; panels are stored one after the other. A
// column is stored with n16 - 16k slots, n16 = n rounded up to a multiple of
// 16, so every column (and every 64-row chunk of one) starts on a 16-entry
// boundary; the padding slots are never read.
constexpr int SYM_P = 16;
__host__ __device__ inline int sym_n16(int n) { return (n + SYM_P - 1) & ~(SYM_P - 1); }
// offset of panel k (its column stride is sym_n16(n) - 16k)
__host__ __device__ inline int64_t sym_panel_off(int n, int k) {
  return int64_t(SYM_P) * k * sym_n16(n) - int64_t(SYM_P * SYM_P / 2) * k * (k - 1);
}
// stored entries (what the smoother reads), sum over panels of (n - 16k) w
__host__ __device__ inline int64_t sym_size(int n) {
  int64_t s = 0;
  for (int c0 = 0; c0 < n; c0 += SYM_P) s += int64_t(n - c0) * (n - c0 < SYM_P ? n - c0 : SYM_P);
  return s;
}
// arena slots of one patch, padding included (a multiple of 16)
__host__ __device__ inline int64_t sym_arena(int n) {
  if (n <= 0) return 0;
  const int t = (n + SYM_P - 1) / SYM_P, w = n - SYM_P * (t - 1);
  return sym_panel_off(n, t - 1) + int64_t(SYM_P) * w;
}
// Work items of the symmetric GEMV: (64-row chunk R, panel k) for every
// panel with a row in the chunk, k <= min(4R + 3, panels - 1).
__host__ __device__ inline int sym_items(int n) {
  const int t = (n + SYM_P - 1) / SYM_P, nr = (n + 63) / 64;
  int items = 0;
  for (int R = 0; R < nr; ++R) items += (4 * R + 4 < t ? 4 * R + 4 : t);
  return items;
}

// One explicit patch as the device kernels see it.
struct PatchRec {
  int32_t n;        // unknowns in the patch
  int32_t id;       // explicit patch index within its level
  int64_t slot;     // offset into slot_dof / delta
  int64_t fac;      // element offset into the factor arena of its precision
};

// Patch factorisations of one level in flight: records and device scratch.
struct FactorPending {
  int ne = 0;
  int64_t std_slot = 0;
  std::vector<PatchRec> exp_only, std_only;
  double *work = nullptr, *rs = nullptr, *cs = nullptr, *kap = nullptr;
  int32_t *sig = nullptr, *rowp = nullptr, *sts = nullptr, *slot_all = nullptr;
  PatchRec *d_exp = nullptr, *d_std = nullptr, *d_all = nullptr;
};

// An explicit patch in a multiplicative phase: precision picks the arena.
struct MultRec {
  int32_t n;
  int32_t f32;      // 1: factor in the FP32 arena
  int64_t slot;
  int64_t fac;
};

// One workgroup of the cooperative phase form: the patch record, the first of
// its rows, and the index of its arrival counter (one load per workgroup).
struct CoopItem {
  MultRec rec;
  int32_t r0;
  int32_t cnt;
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
  uint8_t* d_emask = nullptr;     // per cell: bit 0 / bit 1 = its u / v row has E_E entries
  int32_t* d_erow_ptr = nullptr;  // n_erows + 1
  int32_t* d_ecol = nullptr;
  double* d_eval = nullptr;       // -dt * E_E
  // device: full row pointer (2N^2+1) into the same col/val arrays, for patch assembly
  int32_t* d_erow_full = nullptr;

  // patches (levels >= 1)
  bool has_patches = false;
  std::vector<uint8_t> cellflag;           // bit0 explicit seed, bit1 covered, bits 2/3/4: the cell's u/v/p is touched
  std::vector<int64_t> patch_off;          // all patches (N^2 + 1), for export
  std::vector<int32_t> patch_dofs;
  std::vector<int32_t> exp_cells;          // explicit patch -> seed cell
  std::vector<int64_t> exp_off;            // explicit patch -> slot offset (n_exp + 1)
  std::vector<int64_t> exp_cov_off;        // explicit patch -> offset into exp_cov (n_exp + 1)
  std::vector<int32_t> exp_cov;            // cells C_e whose unknowns make up patch e (host only)
  std::vector<int32_t> slot_dof_h;
  std::vector<uint8_t> slot_mask_h;        // box family: 1 where the slot's unknown is injected
  uint8_t* d_slot_mask = nullptr;           // nullptr for the CAV / Vanka families
  uint8_t* d_cellflag = nullptr;
  int32_t n_exp = 0;
  int64_t n_slots = 0;
  int32_t* d_slot_dof = nullptr;
  int2* d_slot_q = nullptr;                // per slot: E_E entry range [x, y) of its unknown (empty for p)
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
  std::vector<int64_t> pred_ptr;          // explicit patch id -> offsets into pred (n_exp + 1)
  std::vector<int32_t> pred;              // conflicting patches of earlier colours (explicit ids)
  MultRec* d_mrec = nullptr;              // records in ph_exp order
  int32_t mrec_max_n = 0;
  std::vector<double> ph_bytes;           // algorithmic bytes of each phase launch
  std::vector<int32_t> ph_maxn;           // largest patch of each phase
  int32_t smoother = -1;                  // per-level smoother kind (-1: the context's)
  double alpha = 0.0;                     // its damping when smoother >= 0
  int32_t mx_nt[4] = {3, 3, 3, 3};              // per size bucket: 256/512/1024 threads, 0 = split form,
                                                // 1/2 = cooperative form with 64/128 rows per workgroup,
                                                // 3 = cooperative form with a shared residual (autotuned)
  int32_t* d_ph_ptr = nullptr;            // device copy of ph_ptr (persistent sweep)
  // explicit phases of a sweep: 0 one launch per phase (default), 1 one
  // cooperative launch with a grid barrier per phase, 2 one dataflow launch
  int sweep_mode = 0;
  // dataflow sweep: per phase-order patch its successors (patches of later
  // colours that conflict with it; d_pr_ptr holds n + 1 offsets, then the
  // item completions each patch waits for per sweep) and the successor list
  // (int32, in d_pr); the ticket counter and per-patch arrival counters
  // (flow[0] ticket, flow[1 + p] completions signalled to patch p), both
  // monotonic: the host keeps the ticket base and the sweep index of the next launch
  int32_t* d_pr_ptr = nullptr;
  int32_t* d_pr = nullptr;
  unsigned long long* d_flow = nullptr;
  uint64_t flow_base = 0, flow_sweep = 0;
  int flow_grid = 0;
  int64_t flow_items = 0;
  double flow_bytes = 0;                  // algorithmic bytes of one dataflow sweep
  int sweep_grid = 0;                     // its workgroups (0: not yet computed)
  std::vector<int32_t> ph_wptr;           // split form: work items of each phase (offsets)
  int2* d_wrk = nullptr;                  // (record index in d_mrec, first row)
  size_t sp_lds = 0;                      // dynamic LDS of the split GEMV kernel
  size_t mx_lds = 0;                      // dynamic LDS of the phase kernel
  // cooperative phase form: items of 64- and 128-row blocks per phase (the
  // 64-row form has the split form's item offsets ph_wptr), arrival counters
  // (records of the 64-row form, then of the 128-row form), and its LDS
  std::vector<int32_t> ph_wptr2;
  CoopItem* d_citem[2] = {nullptr, nullptr};
  int4* d_irow = nullptr;                 // 64 rows per 64-row item: unknown (-1 past the patch), E_E range
  unsigned long long* d_pcnt = nullptr;
  size_t cp_lds[2] = {0, 0};
  size_t mr_lds = 0;                      // multi-RHS phase kernel: n x 16 residual block
  // factorisations enqueued while the host still builds the patch tables
  FactorPending fpend;
  bool fpending = false;
  int cr_pf = 0;                          // shared-residual form: LDS bytes for the prefetched GEMV slice
  size_t cr_lds = 0;                      // and its whole dynamic LDS

  // factors
  bool factored = false;
  double* d_std_inv = nullptr;            // 25 doubles, role order (u_l, u_r, v_b, v_t, p)
  std::vector<PatchRec> rec64_h, rec32_h; // sorted by n descending
  PatchRec* d_rec64 = nullptr;
  PatchRec* d_rec32 = nullptr;
  double* d_f64 = nullptr;
  float* d_f32 = nullptr;
  double bytes64 = 0, bytes32 = 0;        // algorithmic bytes of one GEMV launch per precision
  bool packed = false;                    // inverses in the symmetric panel layout
  bool coloured = false;                  // ph_ptr / ph_exp / pred hold this patch set's colour phases

  // per-level vectors (3 N^2)
  double *d_b = nullptr, *d_x = nullptr, *d_r = nullptr, *d_z = nullptr;
  // 16-column blocks (column stride 3 N^2) of the multi-RHS cycle, made on first use
  double *d_mb = nullptr, *d_mx = nullptr, *d_mr = nullptr;
  double* d_part = nullptr;               // reduction partials
};

// Learned correction stage: 3x3 periodic conv net 3 -> 32 -> 32 -> 3 (no biases).
constexpr int NET_CH = 32;
constexpr int NET_W = 32 * 3 * 9 + 32 * 32 * 9 + 3 * 32 * 9;  // 10 944 master weights
// packed bf16-rounded float layouts used by the kernels (offsets into Net::d_pk)
constexpr int PK_L1F = 0;                 // layer 1 forward  [a][c][ci][co]  9 x 3 x 32
constexpr int PK_L2T = PK_L1F + 864;      // layer 2 backward [a][c][co][ci]  9 x 32 x 32
constexpr int PK_L3F = PK_L2T + 9216;     // layer 3 forward  [a][c][ci][co]  9 x 32 x 3
constexpr int PK_L3T = PK_L3F + 864;      // layer 3 backward [a][c][co][ci]  9 x 3 x 32
constexpr int PK_TOTAL = PK_L3T + 864;

struct Net {
  int device = 0;
  hipStream_t stream = nullptr;
  std::string err;
  float* d_w = nullptr;          // master weights (FP32), flat: W1 (32,3,3,3), W2 (32,32,3,3), W3 (3,32,3,3)
  float* d_g = nullptr;          // gradient of the last training step
  float* d_m = nullptr;          // Adam moments
  float* d_v = nullptr;
  int64_t adam_t = 0;
  float* d_pk = nullptr;         // PK_TOTAL floats
  uint16_t* d_w2m = nullptr;     // layer 2 for the matrix-core kernel: bf16 [co][(a*3+c)*32+ci]
  int64_t cap_pix = 0;           // pixels (batch x N^2) the activation buffers hold
  uint16_t* d_a1 = nullptr;      // NHWC bf16, 32 channels
  uint16_t* d_a2 = nullptr;
  float* d_y3 = nullptr;         // [b][3][N][N]
  float* d_g3 = nullptr;         // [b][3][N][N]
  float* d_g2 = nullptr;         // NHWC FP32
  float* d_g1 = nullptr;
  float* d_wpart = nullptr;      // weight-gradient partials
  int64_t wpart_cap = 0;
  double* d_ls = nullptr;        // loss partials and per-sample sums
  int64_t ls_cap = 0;
  int32_t* d_idx = nullptr;
  int idx_cap = 0;
  double* d_red = nullptr;       // reductions of the FP64 stage (norms)
  int64_t red_cap = 0;
  double* d_rl = nullptr;        // residual-loss workspace: r, c, res, K res (4 x 3N^2) + partials
  int64_t rl_n = 0;
  std::vector<void*> allocs;
  cav_allocator ua{};            // the caller's allocator (cav_net_create), if any
  bool has_ua = false;
};

// Device-resident FGMRES state (graph mode). Integer slots:
enum { GI_J = 0, GI_DONE = 1, GI_K = 2, GI_CONV = 3, GI_COUNT = 4 };
// Double slots: beta, estimate, 1/h_{j+1,j}, then cs[m], sn[m], g[m+1], hist[m], H[(m+1) x m] (column-major).
enum { GS_BETA = 0, GS_EST = 1, GS_INVHN = 2, GS_CS = 4 };
constexpr int64_t GS_H(int m) { return GS_CS + 4 * int64_t(m) + 1; }
constexpr int64_t GS_SIZE(int m) { return GS_H(m) + int64_t(m + 1) * m; }

// Scratch and result of a coarsest factorisation in flight.
struct CoarsePending {
  double *W = nullptr, *Dv = nullptr, *R = nullptr, *X = nullptr;
  int32_t* sts = nullptr;
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
  bool std_first = true;   // multiplicative sweep: shared-patch colours before the explicit phases
  uint32_t wait_limit = 1u << 21;  // polls of a bounded workgroup-barrier wait before it gives up
  int smoother = CAV_SMOOTHER_ADDITIVE;
  int layout = CAV_LAYOUT_FULL;   // patch-inverse storage of the next factorisation
  // interpolation J and spreading S at the structure positions of the last
  // operator build: per Lagrangian row its 16 faces and kernel weights; per
  // touched velocity face its rows and the weights omega * w / h^2
  // (built on first use from the positions kept here, and kept across
  // operator builds at the same positions)
  bool ib_ready = false;
  int ib_N = 0;
  std::vector<double> ib_X, ib_omega;
  int32_t ib_rows = 0, ib_faces = 0;
  int32_t* d_ib_face = nullptr;
  double* d_ib_w = nullptr;
  int32_t* d_sp_face = nullptr;
  int32_t* d_sp_ptr = nullptr;
  int32_t* d_sp_row = nullptr;
  double* d_sp_w = nullptr;
  // coarsest solution operator (nc x nc, row-major, nc = 3 N0^2)
  int nc = 0;
  double* d_cinv = nullptr;
  // FGMRES workspace
  int ws_maxit = 0;
  int64_t ws_n = 0;  // vector length the workspace was sized for
  double *d_V = nullptr, *d_Z = nullptr, *d_w = nullptr, *d_bb = nullptr;
  double *d_h = nullptr, *d_part = nullptr;
  double* h_pinned = nullptr;
  std::vector<void*> allocs;
  // learned stage (not owned) and its workspace
  Net* net = nullptr;
  double net_margin = 1e-3;
  double* d_st = nullptr;        // r', c, K c (3 n)
  double* d_sc = nullptr;        // stage scalars and counters
  int64_t st_n = 0;
  double *d_pw = nullptr;        // residual-pair workspace (5 x 16 columns, 16 norms, partials)
  int64_t pw_n = 0;
  // graph-mode FGMRES: own stream (capture needs a non-default stream),
  // device state, fixed V-cycle input/output, captured iteration body
  unsigned long long* d_bar = nullptr;   // persistent-sweep barrier counter and error flag (2 x u64)
  bool capturing = false;                // set while a graph is being captured
  hipStream_t gstream = nullptr;
  hipStream_t side = nullptr;            // default-priority stream for the coarsest factorisation
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  // stream of the patch factorisations enqueued by the patch build, so that
  // the build's own uploads on `stream` do not queue behind them
  hipStream_t fstream = nullptr;
  hipEvent_t ev_fup = nullptr, ev_fdone = nullptr, ev_fdone2 = nullptr;
  hipEvent_t ev_js[2] = {nullptr, nullptr};  // side streams joined into `stream` before a block is returned
  bool fwait = false;                     // `stream` must wait for ev_fdone and ev_fdone2 before reading their results
  // the coarsest factorisation starts when the operator is built (it needs
  // nothing else) and is collected by cav_factor_patches
  CoarsePending coarse_pend;
  bool coarse_pending = false;            // launched on `side`, not yet checked
  bool coarse_ready = false;              // d_cinv holds the current operator's inverse
  int32_t* d_gi = nullptr;
  double* d_gs = nullptr;
  double* d_vin = nullptr;
  double* d_zout = nullptr;
  int g_maxit = 0;
  int64_t g_n = 0;
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
  uint64_t generation = 1;        // bumped by every setup call; a captured body is valid for one generation
  uint64_t graph_generation = 0;
  double graph_rtol = -1.0;
  // live timing of the explicit-patch GEMV and of whole V-cycles (HIP events)
  bool timing = false;
  std::vector<hipEvent_t> ev_pool;
  size_t ev_used = 0;
  struct KtMark {
    int ev;          // event index of the start (the end is ev + 1)
    double bytes;    // algorithmic bytes of the bracketed launches
    int launches;    // launches inside the bracket
    int coop;        // 1: cooperative-form phase launches (64/128 rows), 2: shared-residual form,
                     // 3: dataflow sweep launches
  };
  std::vector<KtMark> kt_marks;
  std::vector<std::pair<int, int>> vc_marks;      // event indices around each V-cycle
};

hipEvent_t next_event(Ctx& c);
inline void timing_begin(Ctx& c, hipStream_t s, int coop = 0) {
  if (!c.timing) return;
  hipEvent_t e = next_event(c);
  c.kt_marks.push_back({int(c.ev_used - 1), 0.0, 0, coop});
  (void)hipEventRecord(e, s);
}
inline void timing_end(Ctx& c, hipStream_t s, double bytes, int launches = 1) {
  if (!c.timing) return;
  hipEvent_t e = next_event(c);
  c.kt_marks.back().bytes = bytes;
  c.kt_marks.back().launches = launches;
  (void)hipEventRecord(e, s);
}

// ---- host setup (setup_host.cpp) ----
struct Structure {
  int M = 0;
  std::vector<double> X, omega;
  HostCSR E;  // 2M x 2M, component interleaved
};
cav_status make_structure(const cav_structure_desc* st, Structure& out, std::string& err);
cav_status fibre_force(const cav_structure_desc* st, std::vector<double>& F, std::string& err);
void ib_supports(int N, const Structure& s, std::vector<int32_t>& face, std::vector<double>& w);
void assemble_ee_finest(int N, const Structure& s, HostCSR& ee);
void galerkin_coarsen(int Nc, const HostCSR& fine, HostCSR& coarse);
void build_patches(int N, const HostCSR& ee, int family, Level& L);
// the two halves of build_patches: the patch sets (all a factorisation
// needs), then the unknown -> slot transpose, weights, colouring and stats
void build_patch_sets(int N, const HostCSR& ee, int family, Level& L);
// colour = false leaves the multiplicative colour phases to a later
// colour_explicit call (they are only read by the multiplicative smoother).
void build_patch_tables(int N, const HostCSR& ee, Level& L, bool colour = true);
void build_box_patches(int N, const HostCSR& ee, int b, int o, Level& L);

// ---- device launches (kernels_*.hip) ----
void launch_apply_op(const Level& L, const double* x, double* y, const double* b, hipStream_t s);
// the Stokes part alone (A_0, G, -D): y = K_0 x, or y = b - K_0 x when b is given
void launch_stencil(const StencilCoef& sc, const double* x, double* y, const double* b, hipStream_t s);
void launch_restrict(const Level& Lf, const double* rf, double* bc, hipStream_t s);
void launch_prolong_add(const Level& Lf, const double* xc, double* xf, hipStream_t s);
// remove_mean = false leaves the pressure mean of the result in place: the
// V-cycle skips it on every smoothing step but the level's last, since K_E
// does not see a constant pressure and the last step removes the whole mean.
void launch_smoother(Ctx& c, Level& L, const double* b, double* x, bool zero_guess, hipStream_t s,
                     bool remove_mean = true);
void launch_mult_smoother(Ctx& c, Level& L, const double* b, double* x, bool zero_guess, hipStream_t s,
                          bool remove_mean = true);
void launch_smoother_multi(Ctx& c, Level& L, const double* b, double* x, int64_t ldv, int kb, bool zero_guess,
                           hipStream_t s, bool remove_mean = true);
void prepare_mult_smoother(size_t lds);
// the whole multiplicative sweep of level L in one cooperative launch; false if not possible
bool launch_mult_sweep(Ctx& c, Level& L, const double* b, double* x, hipStream_t s);
void launch_clear_sweep_flags(Ctx& c, hipStream_t s);
// the explicit phases of a sweep of level L as one dataflow launch; false if not possible
bool launch_mult_flow(Ctx& c, Level& L, const double* b, double* x, hipStream_t s);
void reset_sweep_counters(Ctx& c, hipStream_t s);
void launch_zero_u64(unsigned long long* v, int64_t n, hipStream_t s);
inline int level_smoother(const Ctx& c, const Level& L) { return L.smoother >= 0 ? L.smoother : c.smoother; }
inline double level_alpha(const Ctx& c, const Level& L) { return L.smoother >= 0 ? L.alpha : c.alpha; }
// size bucket of a phase by its largest patch: <= 64, <= 128, <= 256, larger
inline int mx_bucket(int n) { return n <= 64 ? 0 : n <= 128 ? 1 : n <= 256 ? 2 : 3; }
// one explicit phase: nt = 256, 512 or 1024 threads per patch, or 0 for the split form
void launch_mult_phase(Ctx& c, Level& L, int ph, int nt, const double* b, double* x, hipStream_t s);
void launch_fill(double* x, double v, int64_t n, hipStream_t s);
void colour_explicit(int N, const HostCSR& ee, Level& L);
void launch_coarse_solve(const Ctx& c, const double* b, double* x, hipStream_t s);
// Patch factorisation of one smoothed level in two halves: `launch` uploads
// the records on c.stream, enqueues the factorisations on stream ks (after
// the uploads) and returns their scratch; `finish` reads the
// condition estimates back (synchronising), splits the precisions, writes the
// stored inverses and the smoother tables, and releases the scratch. Every
// level's launch can precede every finish, so the GPU factors all levels
// back to back. `release` frees a pending level's scratch after a failure.
FactorPending factor_level_launch(Ctx& c, Level& L, hipStream_t ks);
void factor_level_finish(Ctx& c, Level& L, FactorPending& fp, int precision, double cond_threshold,
                         cav_factor_stats* st);
void factor_level_release(Ctx& c, FactorPending& fp);
// Coarsest factorisation on stream s (assembly, blocked quasi-definite
// Gauss-Jordan, mean fix); `finish` synchronises s, checks the pivots and
// installs the inverse (on a zero pivot it releases everything and throws).
CoarsePending factor_coarse_launch(Ctx& c, hipStream_t s);
void factor_coarse_finish(Ctx& c, CoarsePending& cp, hipStream_t s);
void factor_coarse_release(Ctx& c, CoarsePending& cp);

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
// Synchronise the device; memory released before this is reused from then on.
void device_sync_epoch(Ctx& c);

// learned stage (kernels_learned.hip)
void net_alloc(Net& n, int64_t pix);
void* net_dev_alloc(Net& n, size_t bytes);
void net_dev_free(Net& n, void* p);
void net_pack(Net& n, hipStream_t s);
void net_forward_f32(Net& n, int N, int B, const float* in, const int32_t* idx, float* out, hipStream_t s);
// c = ||r|| N(r / ||r||) with the pressure mean of c removed; nrm2 = device ||r||^2 (one double)
void net_correct_f64(Net& n, int N, const double* r, const double* nrm2, double* c, double* part, hipStream_t s);
void net_train_step(Net& n, int N, int B, const float* rhat, const float* ehat, const int32_t* idx, double lr,
                    double* loss, hipStream_t s);
void net_forward_train(Net& n, int N, int B, const float* rhat, const int32_t* idx, hipStream_t s);
void net_backward_update(Net& n, int N, int B, const float* rhat, const int32_t* idx, double lr, hipStream_t s);
double* net_loss_sums(Net& n, int B);  // 2B doubles: per sample {||res||^2, ||r||^2}
const int32_t* net_upload_index(Net& n, const int32_t* index, int batch, int64_t n_samples, hipStream_t s);
void launch_sample_f64(const float* src, const int32_t* idx, int b, int64_t n3, double* dst, hipStream_t s);
void launch_scaled_f32(const double* q, const double* sums, double coef, int64_t n3, float* dst, hipStream_t s);
void launch_mr_scalars(double* sums, int B, hipStream_t s);
void launch_coef_f32(const double* q, const double* sums, int64_t n3, float* dst, hipStream_t s);
void launch_sub_gamma(double* y, const double* x, const double* z, const double* sums, int64_t n3, hipStream_t s);
// graph-mode FGMRES (kernels_krylov.hip)
void launch_gstate_init(int32_t* gi, double* gs, double beta, int max_it, hipStream_t s);
void launch_col_get(const double* V, int64_t ldv, const int32_t* gi, double* out, int64_t n, hipStream_t s);
void launch_arnoldi_dk(const Level& F, double* V, double* Z, int64_t n, const int32_t* gi_c, int32_t* gi, double* gs,
                       const double* zout, double* w, double* part, double* hd, int max_it, double rtol,
                       hipStream_t s);
void launch_pair_write(const double* r, const double* e, const double* nrm2, float* rhat, float* ehat, int64_t n,
                       hipStream_t s);
void launch_stage_decide(const double* sc, double margin, double* gamma_out, double* counters, hipStream_t s);
void launch_axpy_dev(double* y, const double* a, const double* x, int64_t n, hipStream_t s);

}  // namespace cav

struct cav_net_s {
  cav::Net n;
};

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
// The multiplicative kernels read full column-major patch inverses.
inline void require_full_layout(const Level& L) {
  if (L.packed)
    throw StatusError(CAV_ERR_INVALID_ARG,
                      "the multiplicative smoother reads full patch inverses: set CAV_LAYOUT_FULL and factor again");
}
}  // namespace cav
