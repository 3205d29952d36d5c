// C ABI: context lifecycle, setup orchestration, V-cycle and FGMRES.
#include <algorithm>
#include <exception>
#include <thread>
#include <cmath>
#include <cstring>
#include <new>
#include <functional>
#include <mutex>
#include <unordered_map>

#include "cav_internal.hpp"

struct cav_ctx_s {
  cav::Ctx c;
  std::unordered_map<void*, size_t> live;  // device blocks handed out, with their sizes
  // released blocks kept for reuse, by size, each with the epoch of its release
  std::unordered_multimap<size_t, std::pair<void*, uint64_t>> cache;
  size_t cached_bytes = 0;
  uint64_t epoch = 1;                      // advanced by every device-wide synchronisation
  // the caller's allocator (cav_create); without it the context calls hipMalloc
  cav_allocator ua{};
  bool has_ua = false;
  int64_t n_hip_malloc = 0, n_ua_alloc = 0, n_ua_free = 0;
};

namespace cav {

static cav_ctx_s* owner(Ctx& c) { return reinterpret_cast<cav_ctx_s*>(&c); }

// Fixed device scratch of cav_fgmres_solve_noalloc: the FGMRES workspace for
// callers that cannot allocate. Every device the library runs on holds its
// own copy until the process ends. Host code never uses the array's name as
// an address: cav_create looks the device address up once per device (with
// that device current) and the entry point passes that address on.
constexpr size_t NOALLOC_SCRATCH_DOUBLES = size_t(1) << 26;  // 512 MiB
static __device__ __align__(256) double scratch[NOALLOC_SCRATCH_DOUBLES];
constexpr int NOALLOC_MAX_DEVICES = 64;
static std::mutex g_scratch_mu;
static double* g_scratch_ptr[NOALLOC_MAX_DEVICES];
static bool g_scratch_looked[NOALLOC_MAX_DEVICES];

// Looks up the scratch's device address on `device`, which must be current.
static hipError_t noalloc_lookup(int device) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (device < 0 || device >= NOALLOC_MAX_DEVICES) return hipSuccess;
  if (g_scratch_looked[device]) return hipSuccess;
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return e;
  }
  g_scratch_ptr[device] = static_cast<double*>(p);
  g_scratch_looked[device] = true;
  return hipSuccess;
}

// The device address of `device`'s scratch, or nullptr if it is not known.
static double* noalloc_scratch(int device) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (device < 0 || device >= NOALLOC_MAX_DEVICES) return nullptr;
  return g_scratch_ptr[device];
}

// Device memory of a context, from hipMalloc or from the caller's allocator.
// Released blocks stay with the context (up to DEV_CACHE_CAP bytes) and are
// handed out again for a request of the same rounded size, so rebuilding a
// hierarchy of the same shape allocates nothing; they go back to their source
// when the context is destroyed or an allocation fails. A block released after the last device-wide synchronisation
// (device_sync_epoch) may still be used by queued work on some stream, so only
// blocks released before it are handed out; the setup calls synchronise once
// after releasing the previous hierarchy's memory.
constexpr size_t DEV_CACHE_CAP = size_t(8) << 30;

// Orders the work queued on the context's side streams before later work on
// its main stream (before a block goes back to a stream-ordered allocator).
static void join_side_streams(Ctx& c) {
  if (!c.side) return;
  CAV_HIP(hipEventRecord(c.ev_js[0], c.side));
  CAV_HIP(hipStreamWaitEvent(c.stream, c.ev_js[0], 0));
  CAV_HIP(hipEventRecord(c.ev_js[1], c.fstream));
  CAV_HIP(hipStreamWaitEvent(c.stream, c.ev_js[1], 0));
}

static void ua_release(cav_ctx_s* o, void* p) {
  o->ua.free(p, static_cast<void*>(o->c.stream), o->ua.user);
  ++o->n_ua_free;
}

// Gives every cached block back to its source (hipFree or the caller's allocator).
static void release_cache(cav_ctx_s* o) {
  if (o->has_ua && !o->cache.empty()) {
    (void)hipDeviceSynchronize();
    for (auto& kv : o->cache) ua_release(o, kv.second.first);
  } else {
    for (auto& kv : o->cache) (void)hipFree(kv.second.first);
  }
  o->cache.clear();
  o->cached_bytes = 0;
}

void* dev_alloc(Ctx& c, size_t bytes) {
  cav_ctx_s* o = owner(c);
  const size_t sz = (std::max<size_t>(bytes, 16) + 255) & ~size_t(255);
  if (!c.capturing) {
    auto r = o->cache.equal_range(sz);
    for (auto it = r.first; it != r.second; ++it)
      if (it->second.second < o->epoch) {
        void* p = it->second.first;
        o->cache.erase(it);
        o->cached_bytes -= sz;
        o->live.emplace(p, sz);
        return p;
      }
  }
  void* p = nullptr;
  if (o->has_ua) {
    p = o->ua.alloc(sz, static_cast<void*>(c.stream), o->ua.user);
    if (!p && !o->cache.empty()) {
      release_cache(o);
      p = o->ua.alloc(sz, static_cast<void*>(c.stream), o->ua.user);
    }
    if (!p) throw StatusError(CAV_ERR_OUT_OF_MEMORY, "the caller's allocator returned no block of " +
                                                         std::to_string(sz) + " bytes");
    ++o->n_ua_alloc;
    o->live.emplace(p, sz);
    return p;
  }
  hipError_t e = hipMalloc(&p, sz);
  ++o->n_hip_malloc;
  if (e != hipSuccess && !o->cache.empty()) {
    (void)hipGetLastError();
    release_cache(o);
    e = hipMalloc(&p, sz);
    ++o->n_hip_malloc;
  }
  if (e != hipSuccess) {
    (void)hipGetLastError();
    throw StatusError(CAV_ERR_OUT_OF_MEMORY, "hipMalloc of " + std::to_string(bytes) + " bytes failed");
  }
  o->live.emplace(p, sz);
  return p;
}

// The context's two extra streams (default priority) and their events.
void ensure_aux_streams(Ctx& c) {
  if (c.side) return;
  CAV_HIP(hipStreamCreateWithFlags(&c.side, hipStreamNonBlocking));
  CAV_HIP(hipStreamCreateWithFlags(&c.fstream, hipStreamNonBlocking));
  for (hipEvent_t* e : {&c.ev_fork, &c.ev_join, &c.ev_fup, &c.ev_fdone, &c.ev_fdone2, &c.ev_js[0], &c.ev_js[1]})
    CAV_HIP(hipEventCreateWithFlags(e, hipEventDisableTiming));
}

// Start the coarsest factorisation on the side stream after the work queued
// on c.stream (the operator's upload).
void start_coarse(Ctx& c) {
  ensure_aux_streams(c);
  CAV_HIP(hipEventRecord(c.ev_fork, c.stream));
  CAV_HIP(hipStreamWaitEvent(c.side, c.ev_fork, 0));
  c.coarse_pend = factor_coarse_launch(c, c.side);
  CAV_HIP(hipEventRecord(c.ev_join, c.side));
  c.coarse_pending = true;
}

// Forget the coarsest factorisation (a new operator is coming).
void drop_coarse(Ctx& c) {
  if (c.coarse_pending) {
    (void)hipStreamSynchronize(c.side);
    factor_coarse_release(c, c.coarse_pend);
    c.coarse_pending = false;
  }
  dev_free(c, c.d_cinv);
  c.d_cinv = nullptr;
  c.coarse_ready = false;
}

void device_sync_epoch(Ctx& c) {
  CAV_HIP(hipDeviceSynchronize());
  ++owner(c)->epoch;
}

void dev_free(Ctx& c, void* p) {
  if (!p) return;
  cav_ctx_s* o = owner(c);
  auto it = o->live.find(p);
  if (it == o->live.end()) return;
  const size_t sz = it->second;
  o->live.erase(it);
  if (o->cached_bytes + sz <= DEV_CACHE_CAP) {
    o->cache.emplace(sz, std::make_pair(p, o->epoch));
    o->cached_bytes += sz;
  } else if (o->has_ua) {
    join_side_streams(c);
    ua_release(o, p);
  } else {
    (void)hipFree(p);
  }
}

hipEvent_t next_event(Ctx& c) {
  if (c.ev_used == c.ev_pool.size()) {
    // timing-only events: no system-scope fence (a cache write-back and
    // invalidate) when one is recorded, so the brackets neither cost a flush
    // nor leave the next launch a cold cache; elapsed times are read after a
    // stream synchronisation
    hipEvent_t e;
    CAV_HIP(hipEventCreateWithFlags(&e, hipEventDisableSystemFence));
    c.ev_pool.push_back(e);
  }
  return c.ev_pool[c.ev_used++];
}

namespace {
constexpr int TPB = 256;

__global__ void k_axpby(double* __restrict__ y, double a, const double* __restrict__ x, double b, int64_t n) {
  const int64_t t = int64_t(blockIdx.x) * TPB + threadIdx.x;
  if (t >= n) return;
  y[t] = a * x[t] + (b == 0.0 ? 0.0 : b * y[t]);
}

inline unsigned nblocks(int64_t n) { return unsigned((n + TPB - 1) / TPB); }

template <typename T>
T* upload(Ctx& c, const std::vector<T>& h) {
  if (h.empty()) return nullptr;
  T* d = static_cast<T*>(dev_alloc(c, h.size() * sizeof(T)));
  CAV_HIP(hipMemcpyAsync(d, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice, c.stream));
  return d;
}

void free_ib_tables(Ctx& c) {
  for (void* p : {(void*)c.d_ib_face, (void*)c.d_ib_w, (void*)c.d_sp_face, (void*)c.d_sp_ptr, (void*)c.d_sp_row,
                  (void*)c.d_sp_w})
    dev_free(c, p);
  c.d_ib_face = c.d_sp_face = c.d_sp_ptr = c.d_sp_row = nullptr;
  c.d_ib_w = c.d_sp_w = nullptr;
  c.ib_rows = c.ib_faces = 0;
  c.ib_ready = false;
}

// J as 16 (face, weight) pairs per Lagrangian row; S = h^-2 J^T W grouped by
// face (rows of one face in increasing order), so that spreading is a
// deterministic gather per touched face
void build_ib_tables(Ctx& c) {
  if (c.ib_ready) return;
  Structure S;
  S.M = int(c.ib_omega.size());
  S.X = c.ib_X;
  S.omega = c.ib_omega;
  const int N = c.ib_N;
  std::vector<int32_t> face;
  std::vector<double> w;
  ib_supports(N, S, face, w);
  const int32_t nr = 2 * S.M;
  const double ih2 = double(N) * N;
  std::vector<std::pair<int32_t, int32_t>> fr;  // (face, row)
  fr.reserve(face.size());
  for (int32_t r = 0; r < nr; ++r)
    for (int t = 0; t < 16; ++t) fr.push_back({face[size_t(r) * 16 + t], r * 16 + t});
  std::sort(fr.begin(), fr.end());
  std::vector<int32_t> sf, sptr(1, 0), srow;
  std::vector<double> sw;
  for (size_t q = 0; q < fr.size(); ++q) {
    if (q == 0 || fr[q].first != fr[q - 1].first) {
      if (q > 0) sptr.push_back(int32_t(srow.size()));
      sf.push_back(fr[q].first);
    }
    const int32_t r = fr[q].second / 16;
    srow.push_back(r);
    sw.push_back(w[size_t(fr[q].second)] * S.omega[r / 2] * ih2);
  }
  if (!fr.empty()) sptr.push_back(int32_t(srow.size()));
  c.ib_rows = nr;
  c.ib_faces = int32_t(sf.size());
  c.d_ib_face = upload(c, face);
  c.d_ib_w = upload(c, w);
  c.d_sp_face = upload(c, sf);
  c.d_sp_ptr = upload(c, sptr);
  c.d_sp_row = upload(c, srow);
  c.d_sp_w = upload(c, sw);
  c.ib_ready = true;
}

__global__ void k_ib_interp(int32_t nr, const int32_t* __restrict__ face, const double* __restrict__ w,
                            const double* __restrict__ x, double* __restrict__ U) {
  const int32_t r = int32_t(blockIdx.x) * TPB + int32_t(threadIdx.x);
  if (r >= nr) return;
  double acc = 0.0;
  for (int t = 0; t < 16; ++t) acc += w[int64_t(r) * 16 + t] * x[face[int64_t(r) * 16 + t]];
  U[r] = acc;
}

__global__ void k_ib_spread(int32_t nf, const int32_t* __restrict__ face, const int32_t* __restrict__ ptr,
                            const int32_t* __restrict__ row, const double* __restrict__ w, const double* __restrict__ F,
                            double* __restrict__ y) {
  const int32_t q = int32_t(blockIdx.x) * TPB + int32_t(threadIdx.x);
  if (q >= nf) return;
  double acc = 0.0;
  for (int32_t k = ptr[q]; k < ptr[q + 1]; ++k) acc += w[k] * F[row[k]];
  y[face[q]] += acc;
}

void free_patches(Ctx& c, Level& L);

void free_level(Ctx& c, Level& L) {
  free_patches(c, L);  // every patch-level block, the dataflow tables included
  for (void* p : {(void*)L.d_erow_id, (void*)L.d_erow_ptr, (void*)L.d_ecol, (void*)L.d_eval, (void*)L.d_erow_full,
                  (void*)L.d_emask, (void*)L.d_b, (void*)L.d_x, (void*)L.d_r, (void*)L.d_z, (void*)L.d_part,
                  (void*)L.d_mb, (void*)L.d_mx, (void*)L.d_mr})
    dev_free(c, p);
  L = Level();
}

void free_patches(Ctx& c, Level& L) {
  if (L.fpending) {
    factor_level_release(c, L.fpend);   // blocks are reused only after a device-wide synchronisation
    L.fpending = false;
  }
  for (void** p : {(void**)&L.d_cellflag, (void**)&L.d_slot_dof, (void**)&L.d_delta, (void**)&L.d_t_dof,
                   (void**)&L.d_t_inv, (void**)&L.d_t_ptr, (void**)&L.d_t_slot, (void**)&L.d_std_inv,
                   (void**)&L.d_rec64, (void**)&L.d_rec32, (void**)&L.d_f64, (void**)&L.d_f32,
                   (void**)&L.d_mrec, (void**)&L.d_wrk, (void**)&L.d_ph_ptr, (void**)&L.d_slot_mask,
                   (void**)&L.d_citem[0], (void**)&L.d_citem[1], (void**)&L.d_pcnt,
                   (void**)&L.d_slot_q, (void**)&L.d_irow, (void**)&L.d_pr_ptr, (void**)&L.d_pr,
                   (void**)&L.d_flow}) {
    dev_free(c, *p);
    *p = nullptr;
  }
  L.flow_base = L.flow_sweep = 0;
  L.flow_items = 0;
  L.rec64_h.clear();
  L.rec32_h.clear();
  L.has_patches = false;
  L.factored = false;
}

// The pressure mean is removed once per cycle, at its end on the top level:
// K_E, the smoothers' residuals and the transfers do not see a constant
// pressure (G annihilates it and prolongation keeps means), so the means the
// other smoothing steps and levels leave change nothing else.
void vcycle_level(Ctx& c, int l, const double* b, double* x, bool top = true) {
  hipStream_t s = c.stream;
  if (l == 0) {
    launch_coarse_solve(c, b, x, s);
    return;
  }
  Level& L = c.lv[l];
  const int64_t n = 3 * int64_t(L.N) * L.N;
  if (c.pre == 0) launch_fill(x, 0.0, n, s);
  for (int k = 0; k < c.pre; ++k) launch_smoother(c, L, b, x, k == 0, s, false);
  Level& C = c.lv[l - 1];
  launch_apply_op(L, x, L.d_r, b, s);  // r = b - K x
  launch_restrict(L, L.d_r, C.d_b, s);
  vcycle_level(c, l - 1, C.d_b, C.d_x, false);
  launch_prolong_add(L, C.d_x, x, s);
  for (int k = 0; k < c.post; ++k) launch_smoother(c, L, b, x, false, s, top && k + 1 == c.post);
  if (top && c.post == 0) launch_pressure_mean_remove(x, L.N, L.d_part, s);
}

// The V-cycle on kb <= 16 right-hand sides at once (columns of b and x with
// stride 3 N^2 of level l): the same steps as vcycle_level for every column,
// with the explicit-patch phases of the multiplicative smoother applied to all
// columns in one launch (one read of each stored inverse per phase).
constexpr int MR_COLS = 16;
void vcycle_level_multi(Ctx& c, int l, const double* b, double* x, int kb, bool top = true) {
  hipStream_t s = c.stream;
  const int64_t n = 3 * int64_t(c.lv[l].N) * c.lv[l].N;
  if (l == 0) {
    for (int q = 0; q < kb; ++q) launch_coarse_solve(c, b + q * n, x + q * n, s);
    return;
  }
  Level& L = c.lv[l];
  if (c.pre == 0)
    for (int q = 0; q < kb; ++q) launch_fill(x + q * n, 0.0, n, s);
  for (int k = 0; k < c.pre; ++k) launch_smoother_multi(c, L, b, x, n, kb, k == 0, s, false);
  Level& C = c.lv[l - 1];
  const int64_t nc = 3 * int64_t(C.N) * C.N;
  for (int q = 0; q < kb; ++q) {
    launch_apply_op(L, x + q * n, L.d_mr + q * n, b + q * n, s);  // r = b - K x
    launch_restrict(L, L.d_mr + q * n, C.d_mb + q * nc, s);
  }
  vcycle_level_multi(c, l - 1, C.d_mb, C.d_mx, kb, false);
  for (int q = 0; q < kb; ++q) launch_prolong_add(L, C.d_mx + q * nc, x + q * n, s);
  for (int k = 0; k < c.post; ++k) launch_smoother_multi(c, L, b, x, n, kb, false, s, top && k + 1 == c.post);
  if (top && c.post == 0)
    for (int q = 0; q < kb; ++q) launch_pressure_mean_remove(x + q * n, L.N, L.d_part, s);
}

void ensure_multi_workspace(Ctx& c) {
  for (Level& L : c.lv) {
    if (L.d_mb) continue;
    const size_t bytes = size_t(MR_COLS) * 3 * size_t(L.N) * L.N * sizeof(double);
    L.d_mb = static_cast<double*>(dev_alloc(c, bytes));
    L.d_mx = static_cast<double*>(dev_alloc(c, bytes));
    L.d_mr = static_cast<double*>(dev_alloc(c, bytes));
  }
}

void require(bool ok, cav_status st, const char* msg) {
  if (!ok) throw StatusError(st, msg);
}

// Factored patches, and no multiplicative level over inverses in the
// symmetric panel layout (the multiplicative kernels read full inverses).
void require_factored(const Ctx& c, const char* msg) {
  require(c.factored, CAV_ERR_NOT_BUILT, msg);
  for (int l = 1; l < c.n_levels; ++l)
    require(!c.lv[l].packed || level_smoother(c, c.lv[l]) != CAV_SMOOTHER_MULTIPLICATIVE, CAV_ERR_INVALID_ARG,
            "the multiplicative smoother reads full patch inverses: set CAV_LAYOUT_FULL and factor again");
}

// Top-level V-cycle on the finest level, timed when live timing is on.
void vcycle_top(Ctx& c, const double* r, double* z) {
  int start = -1;
  if (c.timing) {
    hipEvent_t e = next_event(c);
    start = int(c.ev_used - 1);
    CAV_HIP(hipEventRecord(e, c.stream));
  }
  vcycle_level(c, c.n_levels - 1, r, z);
  if (c.timing) {
    hipEvent_t e = next_event(c);
    c.vc_marks.push_back({start, int(c.ev_used - 1)});
    CAV_HIP(hipEventRecord(e, c.stream));
  }
}

void ensure_workspace(Ctx& c, int max_it) {
  const Level& F = c.lv.back();
  const int64_t n = 3 * int64_t(F.N) * F.N;
  if (c.ws_maxit >= max_it && c.ws_n == n && c.d_V) return;
  for (void* p : {(void*)c.d_V, (void*)c.d_Z, (void*)c.d_w, (void*)c.d_bb, (void*)c.d_h, (void*)c.d_part})
    dev_free(c, p);
  if (c.h_pinned) (void)hipHostFree(c.h_pinned);
  c.h_pinned = nullptr;
  c.ws_n = n;
  c.d_V = static_cast<double*>(dev_alloc(c, size_t(max_it + 1) * n * sizeof(double)));
  c.d_Z = static_cast<double*>(dev_alloc(c, size_t(max_it) * n * sizeof(double)));
  c.d_w = static_cast<double*>(dev_alloc(c, size_t(n) * sizeof(double)));
  c.d_bb = static_cast<double*>(dev_alloc(c, size_t(n) * sizeof(double)));
  c.d_h = static_cast<double*>(dev_alloc(c, size_t(3 * (max_it + 2)) * sizeof(double)));
  c.d_part = static_cast<double*>(dev_alloc(c, size_t(dots_blocks(n)) * (max_it + 2) * sizeof(double)));
  CAV_HIP(hipHostMalloc(reinterpret_cast<void**>(&c.h_pinned), size_t(3 * (max_it + 2)) * sizeof(double),
                        hipHostMallocDefault));
  c.ws_maxit = max_it;
}

// ||x||_2 of a device vector (fixed-order reduction over `part`, result in
// h[0]), synchronising.
double dnorm_ws(Ctx& c, const double* x, int64_t n, double* part, double* h) {
  const int nb = dots_blocks(n);
  launch_dots(x, n, 1, x, n, part, nb, h, c.stream);
  double v = 0;
  CAV_HIP(hipMemcpyAsync(&v, h, sizeof(double), hipMemcpyDeviceToHost, c.stream));
  CAV_HIP(hipStreamSynchronize(c.stream));
  return std::sqrt(v);
}
double dnorm(Ctx& c, const double* x, int64_t n) { return dnorm_ws(c, x, n, c.d_part, c.d_h); }

// A persistent sweep whose grid barrier timed out leaves a flag: report it.
void check_sweep_flags(Ctx& c) {
  if (!c.d_bar) return;
  unsigned long long f[2] = {0, 0};
  CAV_HIP(hipMemcpyAsync(f, c.d_bar, sizeof(f), hipMemcpyDeviceToHost, c.stream));
  CAV_HIP(hipStreamSynchronize(c.stream));
  if (f[1] != 0) {
    launch_clear_sweep_flags(c, c.stream);
    reset_sweep_counters(c, c.stream);
    throw StatusError(CAV_ERR_HIP, "a smoother sweep timed out at a workgroup barrier; results are invalid");
  }
}

// ---- graph-mode FGMRES ----
void drop_graph(Ctx& c) {
  if (c.gexec) (void)hipGraphExecDestroy(c.gexec);
  if (c.graph) (void)hipGraphDestroy(c.graph);
  c.gexec = nullptr;
  c.graph = nullptr;
  c.graph_generation = 0;
}

void graph_workspace(Ctx& c, int max_it) {
  ensure_workspace(c, max_it);
  const int64_t n = c.ws_n;
  if (!c.gstream) CAV_HIP(hipStreamCreateWithFlags(&c.gstream, hipStreamNonBlocking));
  if (c.d_gi && c.g_maxit == max_it && c.g_n == n) return;
  drop_graph(c);
  for (void* p : {(void*)c.d_gi, (void*)c.d_gs, (void*)c.d_vin, (void*)c.d_zout}) dev_free(c, p);
  c.d_gi = static_cast<int32_t*>(dev_alloc(c, GI_COUNT * sizeof(int32_t)));
  c.d_gs = static_cast<double*>(dev_alloc(c, size_t(GS_SIZE(max_it)) * sizeof(double)));
  c.d_vin = static_cast<double*>(dev_alloc(c, size_t(n) * sizeof(double)));
  c.d_zout = static_cast<double*>(dev_alloc(c, size_t(n) * sizeof(double)));
  c.g_maxit = max_it;
  c.g_n = n;
}

// One FGMRES iteration of the context's system, enqueued on c.stream; every
// launch reads the iteration index from device memory.
void graph_body(Ctx& c, double rtol) {
  const Level& F = c.lv.back();
  const int64_t n = c.g_n;
  launch_col_get(c.d_V, n, c.d_gi, c.d_vin, n, c.stream);
  vcycle_level(c, c.n_levels - 1, c.d_vin, c.d_zout);
  launch_arnoldi_dk(F, c.d_V, c.d_Z, n, c.d_gi, c.d_gi, c.d_gs, c.d_zout, c.d_w, c.d_part, c.d_h, c.g_maxit, rtol,
                    c.stream);
}

// Capture `bodies` on the streams of the given contexts, forked from and joined
// into `origin`, as one graph.
hipGraphExec_t capture_bodies(const std::vector<Ctx*>& cs, hipStream_t origin, double rtol, hipGraph_t* out_graph) {
  std::vector<hipStream_t> saved;
  std::vector<bool> tsaved;
  for (Ctx* c : cs) {
    saved.push_back(c->stream);
    tsaved.push_back(c->timing);
    c->timing = false;
    c->capturing = true;  // per-phase launches only (no cooperative launch inside a graph)
  }
  hipEvent_t fork;
  CAV_HIP(hipEventCreateWithFlags(&fork, hipEventDisableTiming));
  std::vector<hipEvent_t> joins(cs.size(), nullptr);
  hipGraph_t g = nullptr;
  bool capturing = false;
  try {
    CAV_HIP(hipStreamBeginCapture(origin, hipStreamCaptureModeThreadLocal));
    capturing = true;
    CAV_HIP(hipEventRecord(fork, origin));
    for (size_t i = 0; i < cs.size(); ++i) {
      Ctx& c = *cs[i];
      c.stream = c.gstream == origin ? origin : c.gstream;
      if (c.stream != origin) CAV_HIP(hipStreamWaitEvent(c.stream, fork, 0));
      graph_body(c, rtol);
      if (c.stream != origin) {
        CAV_HIP(hipEventCreateWithFlags(&joins[i], hipEventDisableTiming));
        CAV_HIP(hipEventRecord(joins[i], c.stream));
        CAV_HIP(hipStreamWaitEvent(origin, joins[i], 0));
      }
    }
    capturing = false;
    CAV_HIP(hipStreamEndCapture(origin, &g));
  } catch (...) {
    if (capturing) {
      hipGraph_t junk = nullptr;
      (void)hipStreamEndCapture(origin, &junk);
      if (junk) (void)hipGraphDestroy(junk);
    }
    for (size_t i = 0; i < cs.size(); ++i) {
      cs[i]->stream = saved[i];
      cs[i]->timing = tsaved[i];
      cs[i]->capturing = false;
    }
    (void)hipEventDestroy(fork);
    for (hipEvent_t e : joins)
      if (e) (void)hipEventDestroy(e);
    throw;
  }
  for (size_t i = 0; i < cs.size(); ++i) {
    cs[i]->stream = saved[i];
    cs[i]->timing = tsaved[i];
    cs[i]->capturing = false;
  }
  (void)hipEventDestroy(fork);
  for (hipEvent_t e : joins)
    if (e) (void)hipEventDestroy(e);
  hipGraphExec_t ex = nullptr;
  hipError_t e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    (void)hipGraphDestroy(g);
    throw HipError(std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
  }
  *out_graph = g;
  return ex;
}

// Prologue shared by the graph solves: b' = b minus its pressure mean (into
// d_bb), beta = ||b'||, v_0 = b'/beta, device state reset. Runs on c.stream.
struct Start {
  double beta = 0.0, pmean = 0.0;
};
Start graph_start(Ctx& c, const double* b) {
  hipStream_t s = c.stream;
  const Level& F = c.lv.back();
  const int64_t n = c.g_n, n2 = int64_t(F.N) * F.N;
  Start st;
  CAV_HIP(hipMemcpyAsync(c.d_bb, b, size_t(n) * sizeof(double), hipMemcpyDeviceToDevice, s));
  launch_block_sum(c.d_bb + 2 * n2, n2, c.d_part, c.d_h, s);
  double psum = 0.0;
  CAV_HIP(hipMemcpyAsync(&psum, c.d_h, sizeof(double), hipMemcpyDeviceToHost, s));
  CAV_HIP(hipStreamSynchronize(s));
  st.pmean = psum / double(n2);
  require(std::isfinite(st.pmean), CAV_ERR_INVALID_ARG, "right-hand side is not finite");
  launch_pressure_mean_remove(c.d_bb, F.N, c.d_part, s);
  st.beta = dnorm(c, c.d_bb, n);
  require(std::isfinite(st.beta), CAV_ERR_INVALID_ARG, "right-hand side is not finite");
  if (st.beta > 0.0) {
    k_axpby<<<nblocks(n), TPB, 0, s>>>(c.d_V, 1.0 / st.beta, c.d_bb, 0.0, n);
    launch_gstate_init(c.d_gi, c.d_gs, st.beta, c.g_maxit, s);
  }
  return st;
}

// Epilogue: y = H_k^{-1} g on the host, x = Z_k y, true residual, summary.
cav_status graph_finish(Ctx& c, const Start& st, double* x, double rtol, const cav_fgmres_opts* opts,
                        cav_solve_info* info) {
  hipStream_t s = c.stream;
  const Level& F = c.lv.back();
  const int64_t n = c.g_n;
  const int m = c.g_maxit;
  cav_solve_info inf{};
  inf.pressure_mean_removed = st.pmean;
  if (!(st.beta > 0.0)) {
    launch_fill(x, 0.0, n, s);
    CAV_HIP(hipStreamSynchronize(s));
    inf.converged = 1;
    if (info) *info = inf;
    return CAV_OK;
  }
  int32_t gi[GI_COUNT];
  std::vector<double> gs(size_t(GS_SIZE(m)));
  CAV_HIP(hipMemcpyAsync(gi, c.d_gi, sizeof(gi), hipMemcpyDeviceToHost, s));
  CAV_HIP(hipMemcpyAsync(gs.data(), c.d_gs, gs.size() * sizeof(double), hipMemcpyDeviceToHost, s));
  CAV_HIP(hipStreamSynchronize(s));
  if (gi[GI_DONE] == 2) throw StatusError(CAV_ERR_INVALID_ARG, "non-finite value in FGMRES (check inputs)");
  const int k = gi[GI_K];
  const double* H = gs.data() + GS_H(m);
  const double* g = gs.data() + GS_CS + 2 * m;
  const double* hist = g + (m + 1);
  std::vector<double> y(size_t(std::max(k, 1)), 0.0);
  for (int i = k - 1; i >= 0; --i) {
    double acc = g[i];
    for (int q = i + 1; q < k; ++q) acc -= H[int64_t(q) * (m + 1) + i] * y[q];
    y[i] = acc / H[int64_t(i) * (m + 1) + i];
  }
  if (opts && opts->history)
    for (int j = 0; j < k; ++j) opts->history[j] = hist[j];
  CAV_HIP(hipMemcpyAsync(c.d_h, y.data(), size_t(k) * sizeof(double), hipMemcpyHostToDevice, s));
  launch_fill(x, 0.0, n, s);
  launch_multi_axpy(x, c.d_Z, n, k, c.d_h, 1.0, n, s);
  launch_apply_op(F, x, c.d_w, c.d_bb, s);
  const double rn = dnorm(c, c.d_w, n);
  check_sweep_flags(c);
  inf.iterations = k;
  inf.converged = gi[GI_CONV];
  inf.est_rel_residual = gs[GS_EST];
  inf.true_rel_residual = rn / st.beta;
  if (info) *info = inf;
  if (!inf.converged) return CAV_WARN_NOT_CONVERGED;
  if (inf.true_rel_residual > 10.0 * rtol) return CAV_WARN_FLOOR_LIMITED;
  return CAV_OK;
}

// Runs `fn` with c.stream switched to the context's own capture-capable stream,
// ordered after the caller's stream and before its later work.
template <typename Fn>
auto on_graph_stream(Ctx& c, Fn fn) -> decltype(fn()) {
  if (!c.gstream) CAV_HIP(hipStreamCreateWithFlags(&c.gstream, hipStreamNonBlocking));
  hipStream_t caller = c.stream;
  hipEvent_t e;
  CAV_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
  CAV_HIP(hipEventRecord(e, caller));
  CAV_HIP(hipStreamWaitEvent(c.gstream, e, 0));
  c.stream = c.gstream;
  struct Restore {
    Ctx& c;
    hipStream_t caller;
    hipEvent_t e;
    ~Restore() {
      (void)hipEventRecord(e, c.gstream);
      (void)hipStreamWaitEvent(caller, e, 0);
      (void)hipEventDestroy(e);
      c.stream = caller;
    }
  } restore{c, caller, e};
  return fn();
}

// Stage workspace: r', c, K c (3 n doubles) and 8 scalars
// {||r'||^2, <r', Kc>, ||Kc||^2, gamma, accepted, rejected, -, -}.
void ensure_stage_workspace(Ctx& c) {
  const Level& F = c.lv.back();
  const int64_t n = 3 * int64_t(F.N) * F.N;
  if (c.d_st && c.st_n == n) return;
  dev_free(c, c.d_st);
  dev_free(c, c.d_sc);
  c.d_st = static_cast<double*>(dev_alloc(c, size_t(3 * n) * sizeof(double)));
  c.d_sc = static_cast<double*>(dev_alloc(c, 8 * sizeof(double)));
  c.st_n = n;
}

// Learned correction after z0 = V(v): r' = v - K z0, c = ||r'|| N(r'/||r'||)
// (pressure mean removed), gamma = <r', Kc>/||Kc||^2; z0 += gamma c when the
// stage cuts ||r'||^2 by at least the margin, else z0 is kept. All on device.
void learned_stage(Ctx& c, const double* v, double* z, int nbk) {
  const Level& F = c.lv.back();
  hipStream_t s = c.stream;
  const int64_t n = 3 * int64_t(F.N) * F.N;
  double* rp = c.d_st;
  double* cc = c.d_st + n;
  double* kc = c.d_st + 2 * n;
  launch_apply_op(F, z, rp, v, s);
  launch_dots(rp, n, 1, rp, n, c.d_part, nbk, c.d_sc, s);
  net_correct_f64(*c.net, F.N, rp, c.d_sc, cc, c.d_part, s);
  launch_apply_op(F, cc, kc, nullptr, s);
  launch_dots(kc, n, 1, rp, n, c.d_part, nbk, c.d_sc + 1, s);
  launch_dots(kc, n, 1, kc, n, c.d_part, nbk, c.d_sc + 2, s);
  launch_stage_decide(c.d_sc, c.net_margin, c.d_sc + 3, c.d_sc + 4, s);
  launch_axpy_dev(z, c.d_sc + 3, cc, n, s);
}


// Workspace of one FGMRES solve: the Krylov bases V ((m + 1) n doubles) and
// Z (m n), the operator output w and the projected right-hand side bb (n
// each), the device Hessenberg column h (3 (m + 2)), the dot-product partials
// (dots_blocks(n) (m + 2)), and hh, a host buffer of 3 (m + 2) doubles.
struct KrylovWs {
  double *V, *Z, *w, *bb, *h, *part, *hh;
};

// Arguments shared by the FGMRES entry points; returns max_it.
int check_fgmres_args(const Ctx& c, const double* b, const double* x, const cav_fgmres_opts* opts) {
  require_factored(c, "cav_factor_patches has not succeeded");
  require(b && x && b != x, CAV_ERR_INVALID_ARG, "b and x must be distinct device pointers");
  const double rtol = opts ? opts->rtol : 1e-10;
  const int max_it = opts ? opts->max_it : 150;
  require(max_it >= 1 && max_it <= 10000 && rtol >= 0.0, CAV_ERR_INVALID_ARG, "bad FGMRES options");
  return max_it;
}

// The FGMRES solve of cav_fgmres_solve on a given workspace (Section 5).
cav_status fgmres_core(Ctx& c, const double* b, double* x, const cav_fgmres_opts* opts, cav_solve_info* info,
                       const KrylovWs& ws) {
  const double rtol = opts ? opts->rtol : 1e-10;
  const int max_it = opts ? opts->max_it : 150;
  hipStream_t s = c.stream;
  Level& F = c.lv.back();
  const int64_t n = 3 * int64_t(F.N) * F.N, n2 = int64_t(F.N) * F.N;
  // b' = b with the pressure mean projected out (the range of K_E excludes constant pressure)
  CAV_HIP(hipMemcpyAsync(ws.bb, b, size_t(n) * sizeof(double), hipMemcpyDeviceToDevice, s));
  launch_block_sum(ws.bb + 2 * n2, n2, ws.part, ws.h, s);
  double psum = 0.0;
  CAV_HIP(hipMemcpyAsync(&psum, ws.h, sizeof(double), hipMemcpyDeviceToHost, s));
  CAV_HIP(hipStreamSynchronize(s));
  const double pmean = psum / double(n2);
  require(std::isfinite(pmean), CAV_ERR_INVALID_ARG, "right-hand side is not finite");
  launch_pressure_mean_remove(ws.bb, F.N, ws.part, s);
  CAV_HIP(hipGetLastError());
  const double beta = dnorm_ws(c, ws.bb, n, ws.part, ws.h);
  cav_solve_info inf{};
  if (!(beta > 0.0) || !std::isfinite(beta)) {
    require(std::isfinite(beta), CAV_ERR_INVALID_ARG, "right-hand side is not finite");
    launch_fill(x, 0.0, n, s);
    CAV_HIP(hipStreamSynchronize(s));
    inf.converged = 1;
    if (info) *info = inf;
    return CAV_OK;
  }
  double* V = ws.V;
  double* Z = ws.Z;
  k_axpby<<<nblocks(n), TPB, 0, s>>>(V, 1.0 / beta, ws.bb, 0.0, n);
  const int nbk = dots_blocks(n);
  launch_clear_sweep_flags(c, s);
  const bool learned = opts && opts->use_learned;
  if (learned) {
    require(c.net != nullptr, CAV_ERR_NOT_BUILT, "use_learned is set but no net is attached");
    ensure_stage_workspace(c);
    CAV_HIP(hipMemsetAsync(c.d_sc, 0, 8 * sizeof(double), s));
  }
  std::vector<double> H(size_t(max_it + 1) * max_it, 0.0), cs(max_it), sn(max_it), g(max_it + 1, 0.0);
  auto Hat = [&](int i, int j) -> double& { return H[size_t(j) * (max_it + 1) + i]; };
  g[0] = beta;
  int k = 0;
  bool conv = false;
  double est = 1.0;
  double* hd1 = ws.h;
  double* hd2 = ws.h + (max_it + 2);
  double* hdn = ws.h + 2 * (max_it + 2);
  double* hh = ws.hh;
  for (int j = 0; j < max_it; ++j) {
    double* vj = V + int64_t(j) * n;
    double* zj = Z + int64_t(j) * n;
    vcycle_top(c, vj, zj);
    if (learned) learned_stage(c, vj, zj, nbk);
    double* w = ws.w;
    launch_apply_op(F, zj, w, nullptr, s);
    // CGS2
    launch_dots(V, n, j + 1, w, n, ws.part, nbk, hd1, s);
    launch_multi_axpy(w, V, n, j + 1, hd1, -1.0, n, s);
    launch_dots(V, n, j + 1, w, n, ws.part, nbk, hd2, s);
    launch_multi_axpy(w, V, n, j + 1, hd2, -1.0, n, s);
    launch_dots(w, n, 1, w, n, ws.part, nbk, hdn, s);
    CAV_HIP(hipMemcpyAsync(hh, ws.h, size_t(3 * (max_it + 2)) * sizeof(double), hipMemcpyDeviceToHost, s));
    CAV_HIP(hipStreamSynchronize(s));
    for (int i = 0; i <= j; ++i) Hat(i, j) = hh[i] + hh[(max_it + 2) + i];
    const double hn = std::sqrt(hh[2 * (max_it + 2)]);
    Hat(j + 1, j) = hn;
    for (int i = 0; i < j; ++i) {
      const double a = Hat(i, j), bq = Hat(i + 1, j);
      Hat(i, j) = cs[i] * a + sn[i] * bq;
      Hat(i + 1, j) = -sn[i] * a + cs[i] * bq;
    }
    const double rr = std::hypot(Hat(j, j), Hat(j + 1, j));
    const double cj = rr == 0.0 ? 1.0 : Hat(j, j) / rr, sj = rr == 0.0 ? 0.0 : Hat(j + 1, j) / rr;
    cs[j] = cj;
    sn[j] = sj;
    Hat(j, j) = rr;
    Hat(j + 1, j) = 0.0;
    g[j + 1] = -sj * g[j];
    g[j] = cj * g[j];
    k = j + 1;
    est = std::fabs(g[j + 1]) / beta;
    if (opts && opts->history) opts->history[j] = est;
    if (!std::isfinite(est)) {
      check_sweep_flags(c);   // a smoother wait that gave up is the better report
      throw StatusError(CAV_ERR_INVALID_ARG, "non-finite value in FGMRES (check inputs)");
    }
    if (est <= rtol) { conv = true; break; }
    if (hn == 0.0) { conv = true; break; }
    k_axpby<<<nblocks(n), TPB, 0, s>>>(V + int64_t(j + 1) * n, 1.0 / hn, w, 0.0, n);
  }
  // y = H_k^{-1} g, x = Z_k y
  std::vector<double> y(k, 0.0);
  for (int i = k - 1; i >= 0; --i) {
    double acc = g[i];
    for (int q = i + 1; q < k; ++q) acc -= Hat(i, q) * y[q];
    y[i] = acc / Hat(i, i);
  }
  CAV_HIP(hipMemcpyAsync(ws.h, y.data(), size_t(k) * sizeof(double), hipMemcpyHostToDevice, s));
  launch_fill(x, 0.0, n, s);
  launch_multi_axpy(x, Z, n, k, ws.h, 1.0, n, s);
  // true residual in FP64
  launch_apply_op(F, x, ws.w, ws.bb, s);
  const double rn = dnorm_ws(c, ws.w, n, ws.part, ws.h);
  check_sweep_flags(c);
  inf.iterations = k;
  inf.converged = conv ? 1 : 0;
  inf.est_rel_residual = est;
  inf.true_rel_residual = rn / beta;
  inf.pressure_mean_removed = pmean;
  if (learned) {
    double cnt[2] = {0.0, 0.0};
    CAV_HIP(hipMemcpyAsync(cnt, c.d_sc + 4, sizeof(cnt), hipMemcpyDeviceToHost, s));
    CAV_HIP(hipStreamSynchronize(s));
    inf.learned_accepted = int32_t(cnt[0]);
    inf.learned_rejected = int32_t(cnt[1]);
  }
  if (info) *info = inf;
  if (!conv) return CAV_WARN_NOT_CONVERGED;
  if (inf.true_rel_residual > 10.0 * rtol) return CAV_WARN_FLOOR_LIMITED;
  return CAV_OK;
}

}  // namespace
}  // namespace cav

using namespace cav;

#define API_BEGIN try {
#define API_END                                                  \
  }                                                              \
  catch (const StatusError& e) {                                 \
    ctx->c.err = e.msg;                                          \
    return e.st;                                                 \
  }                                                              \
  catch (const HipError& e) {                                    \
    ctx->c.err = e.msg;                                          \
    return CAV_ERR_HIP;                                          \
  }                                                              \
  catch (const std::bad_alloc&) {                                \
    ctx->c.err = "host allocation failed";                       \
    return CAV_ERR_OUT_OF_MEMORY;                                \
  }

extern "C" {

const char* cav_status_string(cav_status s) {
  switch (s) {
    case CAV_OK: return "ok";
    case CAV_ERR_INVALID_ARG: return "invalid argument";
    case CAV_ERR_OUT_OF_MEMORY: return "out of memory";
    case CAV_ERR_HIP: return "HIP runtime error";
    case CAV_ERR_SINGULAR_PATCH: return "singular patch matrix";
    case CAV_ERR_SINGULAR_COARSE: return "singular coarsest matrix";
    case CAV_ERR_NOT_BUILT: return "stage called before its prerequisites";
    case CAV_WARN_NOT_CONVERGED: return "not converged within max_it";
    case CAV_WARN_FLOOR_LIMITED: return "estimate converged, true residual limited by rounding";
  }
  return "unknown status";
}

const char* cav_last_error(cav_ctx ctx) { return ctx ? ctx->c.err.c_str() : "null context"; }

cav_status cav_create(cav_ctx* out, int device, void* stream, const cav_allocator* allocator) {
  if (!out) return CAV_ERR_INVALID_ARG;
  if (allocator && (!allocator->alloc || !allocator->free)) return CAV_ERR_INVALID_ARG;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return CAV_ERR_INVALID_ARG;
  if (hipSetDevice(device) != hipSuccess) return CAV_ERR_HIP;
  if (noalloc_lookup(device) != hipSuccess) return CAV_ERR_HIP;
  cav_ctx ctx = new (std::nothrow) cav_ctx_s();
  if (!ctx) return CAV_ERR_OUT_OF_MEMORY;
  ctx->c.device = device;
  ctx->c.stream = static_cast<hipStream_t>(stream);
  if (allocator) {
    ctx->ua = *allocator;
    ctx->has_ua = true;
  }
  *out = ctx;
  return CAV_OK;
}

cav_status cav_memory_stats(cav_ctx ctx, cav_memory_info* out) {
  if (!ctx || !out) return CAV_ERR_INVALID_ARG;
  cav_memory_info m{};
  for (auto& kv : ctx->live) m.live_bytes += int64_t(kv.second);
  m.live_blocks = int64_t(ctx->live.size());
  m.cached_bytes = int64_t(ctx->cached_bytes);
  m.hip_malloc_calls = ctx->n_hip_malloc;
  m.allocator_allocs = ctx->n_ua_alloc;
  m.allocator_frees = ctx->n_ua_free;
  *out = m;
  return CAV_OK;
}

cav_status cav_set_stream(cav_ctx ctx, void* stream) {
  if (!ctx) return CAV_ERR_INVALID_ARG;
  ctx->c.stream = static_cast<hipStream_t>(stream);
  return CAV_OK;
}

cav_status cav_destroy(cav_ctx ctx) {
  if (!ctx) return CAV_OK;
  (void)hipSetDevice(ctx->c.device);
  if (ctx->c.stream) (void)hipStreamSynchronize(ctx->c.stream);
  if (ctx->c.gexec) (void)hipGraphExecDestroy(ctx->c.gexec);
  if (ctx->c.graph) (void)hipGraphDestroy(ctx->c.graph);
  if (ctx->c.gstream) {
    (void)hipStreamSynchronize(ctx->c.gstream);
    (void)hipStreamDestroy(ctx->c.gstream);
  }
  for (hipStream_t s : {ctx->c.side, ctx->c.fstream})
    if (s) {
      (void)hipStreamSynchronize(s);
      (void)hipStreamDestroy(s);
    }
  for (hipEvent_t e : {ctx->c.ev_fork, ctx->c.ev_join, ctx->c.ev_fup, ctx->c.ev_fdone, ctx->c.ev_fdone2,
                       ctx->c.ev_js[0], ctx->c.ev_js[1]})
    if (e) (void)hipEventDestroy(e);
  // every stream has finished: the blocks go back to whoever gave them
  if (ctx->has_ua) {
    for (auto& kv : ctx->live) ua_release(ctx, kv.first);
  } else {
    for (auto& kv : ctx->live) (void)hipFree(kv.first);
  }
  release_cache(ctx);
  if (ctx->c.h_pinned) (void)hipHostFree(ctx->c.h_pinned);
  for (hipEvent_t e : ctx->c.ev_pool) (void)hipEventDestroy(e);
  delete ctx;
  return CAV_OK;
}

cav_status cav_build_operator(cav_ctx ctx, const cav_grid_desc* g, const cav_structure_desc* st) {
  if (!ctx) return CAV_ERR_INVALID_ARG;
  Ctx& c = ctx->c;
  ++c.generation;
  API_BEGIN
  require(g != nullptr, CAV_ERR_INVALID_ARG, "grid descriptor is NULL");
  const int N = g->N, L = g->n_levels;
  require(N >= 4 && (N & (N - 1)) == 0, CAV_ERR_INVALID_ARG, "N must be a power of two >= 4");
  require(L >= 1 && L <= 30 && (N >> (L - 1)) >= 4 && ((N >> (L - 1)) << (L - 1)) == N, CAV_ERR_INVALID_ARG,
          "n_levels must leave a coarsest grid of at least 4 x 4 cells");
  require(std::isfinite(g->rho) && g->rho > 0 && std::isfinite(g->mu) && g->mu >= 0 && std::isfinite(g->dt) &&
              g->dt > 0,
          CAV_ERR_INVALID_ARG, "rho, dt must be positive and mu non-negative");
  require(int64_t(3) * N * N < (int64_t(1) << 31), CAV_ERR_INVALID_ARG, "grid too large for 32-bit unknown indices");
  Structure S;
  std::string err;
  const cav_status ss = make_structure(st, S, err);
  if (ss != CAV_OK) throw StatusError(ss, err);
  CAV_HIP(hipSetDevice(c.device));
  drop_coarse(c);
  for (auto& lev : c.lv) free_level(c, lev);
  device_sync_epoch(c);
  c.lv.assign(L, Level());
  c.built = c.patched = c.factored = false;
  c.n_levels = L;
  c.rho = g->rho;
  c.mu = g->mu;
  c.dt = g->dt;
  for (int l = 0; l < L; ++l) {
    Level& lev = c.lv[l];
    lev.N = N >> (L - 1 - l);
    lev.h = 1.0 / lev.N;
    lev.sc.N = lev.N;
    lev.sc.diag = c.rho / c.dt + 4.0 * c.mu / (lev.h * lev.h);
    lev.sc.off = c.mu / (lev.h * lev.h);
    lev.sc.invh = 1.0 / lev.h;
  }
  assemble_ee_finest(N, S, c.lv[L - 1].ee);
  for (int l = L - 1; l >= 1; --l) galerkin_coarsen(c.lv[l - 1].N, c.lv[l].ee, c.lv[l - 1].ee);
  if (!(c.ib_N == N && c.ib_X == S.X && c.ib_omega == S.omega)) {
    free_ib_tables(c);
    c.ib_N = N;
    c.ib_X = S.X;
    c.ib_omega = S.omega;
  }
  for (int l = 0; l < L; ++l) {
    Level& lev = c.lv[l];
    const HostCSR& E = lev.ee;
    require(E.nnz() < (int64_t(1) << 31), CAV_ERR_INVALID_ARG, "E_E too large");
    std::vector<int32_t> rid, rptr(1, 0), full(E.n + 1);
    for (int64_t r = 0; r < E.n; ++r) {
      full[r] = int32_t(E.rowptr[r]);
      if (E.rowptr[r + 1] > E.rowptr[r]) {
        rid.push_back(int32_t(r));
        rptr.push_back(int32_t(E.rowptr[r + 1]));
      }
    }
    full[E.n] = int32_t(E.nnz());
    std::vector<double> sval(E.val.size());
    for (size_t k = 0; k < sval.size(); ++k) sval[k] = -c.dt * E.val[k];
    lev.n_erows = int32_t(rid.size());
    {
      // bit 0 / bit 1: the cell's u / v row has E_E entries
      const int64_t n2 = int64_t(lev.N) * lev.N;
      std::vector<uint8_t> mask(size_t(n2), 0);
      for (int32_t r : rid) mask[size_t(r % n2)] |= uint8_t(r < n2 ? 1 : 2);
      lev.d_emask = upload(c, mask);
    }
    lev.d_erow_id = upload(c, rid);
    lev.d_erow_ptr = upload(c, rptr);
    lev.d_ecol = upload(c, E.col);
    lev.d_eval = upload(c, sval);
    lev.d_erow_full = upload(c, full);
    const int64_t n = 3 * int64_t(lev.N) * lev.N;
    lev.d_b = static_cast<double*>(dev_alloc(c, n * sizeof(double)));
    lev.d_x = static_cast<double*>(dev_alloc(c, n * sizeof(double)));
    lev.d_r = static_cast<double*>(dev_alloc(c, n * sizeof(double)));
    lev.d_z = static_cast<double*>(dev_alloc(c, n * sizeof(double)));
    lev.d_part = static_cast<double*>(dev_alloc(c, 1024 * sizeof(double)));
  }
  CAV_HIP(hipStreamSynchronize(c.stream));
  c.built = true;
  // the coarsest inverse needs only the operator: it is computed on the GPU
  // while the host builds the patch sets
  if (3 * int64_t(c.lv[0].N) * c.lv[0].N <= 4096) start_coarse(c);
  return CAV_OK;
  API_END
}

static cav_status build_family(cav_ctx ctx, int family, int box_b, int box_o, cav_level_stats* out) {
  Ctx& c = ctx->c;
  ++c.generation;
  API_BEGIN
  require(c.built, CAV_ERR_NOT_BUILT, "cav_build_operator has not succeeded");
  require(family == CAV_FAMILY_CAV || family == CAV_FAMILY_VANKA || family == CAV_FAMILY_BOX, CAV_ERR_INVALID_ARG,
          "unknown patch family");
  if (family == CAV_FAMILY_BOX) {
    require(box_b >= 1 && box_o >= 0, CAV_ERR_INVALID_ARG, "box size must be >= 1 and overlap >= 0");
    for (int l = 1; l < c.n_levels; ++l)
      require(c.lv[l].N % box_b == 0, CAV_ERR_INVALID_ARG, "every smoothed grid must be a multiple of the box size");
  }
  CAV_HIP(hipSetDevice(c.device));
  c.family = family;
  c.patched = c.factored = false;
  for (int l = 1; l < c.n_levels; ++l) free_patches(c, c.lv[l]);
  // the levels' host-side patch sets are independent: build them concurrently;
  // then the patch factorisations (which need nothing more) are enqueued on the
  // GPU while the host threads build the transposes, weights and colourings
  {
    auto run_levels = [&](const std::function<void(Level&)>& f, const std::function<void()>& beside) {
      std::vector<std::thread> th;
      std::vector<std::exception_ptr> errs(c.n_levels);
      for (int l = 1; l < c.n_levels; ++l)
        th.emplace_back([&, l] {
          try {
            f(c.lv[l]);
          } catch (...) {
            errs[l] = std::current_exception();
          }
        });
      std::exception_ptr mine;
      try {
        beside();
      } catch (...) {
        mine = std::current_exception();
      }
      for (auto& x : th) x.join();
      if (mine) std::rethrow_exception(mine);
      for (auto& e : errs)
        if (e) std::rethrow_exception(e);
    };
    run_levels(
        [&](Level& L) {
          if (family == CAV_FAMILY_BOX)
            build_box_patches(L.N, L.ee, box_b, box_o, L);
          else
            build_patch_sets(L.N, L.ee, family, L);
        },
        [] {});
    run_levels(
        [&](Level& L) {
          // the colour phases only feed the multiplicative kernels, which
          // need the full layout: under the symmetric one they wait for a
          // full-layout factorisation or a phase export
          if (family != CAV_FAMILY_BOX) build_patch_tables(L.N, L.ee, L, c.layout == CAV_LAYOUT_FULL);
        },
        [&] {
          ensure_aux_streams(c);
          for (int l = c.n_levels - 1; l >= 1; --l) {
            // the finest level on its own stream; the smaller ones on the side
            // stream (behind the coarsest factorisation), beside the finest's tail
            c.lv[l].fpend = factor_level_launch(c, c.lv[l], l == c.n_levels - 1 ? c.fstream : c.side);
            c.lv[l].fpending = true;
          }
          CAV_HIP(hipEventRecord(c.ev_fdone, c.fstream));
          CAV_HIP(hipEventRecord(c.ev_fdone2, c.side));
          c.fwait = true;
        });
  }
  for (int l = 1; l < c.n_levels; ++l) {
    Level& L = c.lv[l];
    if (!L.slot_mask_h.empty()) L.d_slot_mask = upload(c, L.slot_mask_h);
    L.d_cellflag = upload(c, L.cellflag);
    L.d_slot_dof = upload(c, L.slot_dof_h);
    {
      const int64_t nv = 2 * int64_t(L.N) * L.N;
      std::vector<int2> sq(L.slot_dof_h.size());
      for (size_t k = 0; k < sq.size(); ++k) {
        const int64_t d = L.slot_dof_h[k];
        sq[k] = d < nv ? make_int2(int(L.ee.rowptr[d]), int(L.ee.rowptr[d + 1])) : make_int2(0, 0);
      }
      L.d_slot_q = upload(c, sq);
    }
    L.d_delta = static_cast<double*>(dev_alloc(c, size_t(std::max<int64_t>(L.n_slots, 1)) * sizeof(double)));
    L.d_t_dof = upload(c, L.t_dof_h);
    L.d_t_inv = upload(c, L.t_inv_h);
    L.d_t_ptr = upload(c, L.t_ptr_h);
    L.d_t_slot = upload(c, L.t_slot_h);
    L.has_patches = true;
  }
  if (out) {
    for (int l = 0; l < c.n_levels; ++l) {
      out[l] = c.lv[l].stats;
      out[l].N = c.lv[l].N;
    }
  }
  CAV_HIP(hipStreamSynchronize(c.stream));
  c.patched = true;
  return CAV_OK;
  API_END
}

cav_status cav_build_cav_patches(cav_ctx ctx, int family, cav_level_stats* out) {
  if (!ctx) return CAV_ERR_INVALID_ARG;
  if (family == CAV_FAMILY_BOX) {
    ctx->c.err = "use cav_build_box_patches for the box family";
    return CAV_ERR_INVALID_ARG;
  }
  return build_family(ctx, family, 0, 0, out);
}

cav_status cav_build_box_patches(cav_ctx ctx, int b, int o, cav_level_stats* out) {
  if (!ctx) return CAV_ERR_INVALID_ARG;
  return build_family(ctx, CAV_FAMILY_BOX, b, o, out);
}

cav_status cav_factor_patches(cav_ctx ctx, int precision, double cond_threshold, cav_factor_stats* out) {
  if (!ctx) return CAV_ERR_INVALID_ARG;
  Ctx& c = ctx->c;
  ++c.generation;
  API_BEGIN
  require(c.patched, CAV_ERR_NOT_BUILT, "cav_build_cav_patches has not succeeded");
  require(precision == CAV_PREC_FP64 || precision == CAV_PREC_MIXED, CAV_ERR_INVALID_ARG, "unknown precision");
  require(!std::isnan(cond_threshold), CAV_ERR_INVALID_ARG, "cond_threshold is NaN");
  CAV_HIP(hipSetDevice(c.device));
  c.factored = false;
  cav_factor_stats st{};
  // every level's patch factorisation is enqueued (finest first) before the
  // first condition estimates are read; the coarsest factorisation normally
  // started with the operator and is only checked here
  std::vector<FactorPending> pend;
  try {
    if (!c.coarse_pending && !c.coarse_ready) start_coarse(c);
    // factorisations normally enqueued by the patch build (a second call factors again)
    for (int l = c.n_levels - 1; l >= 1; --l) {
      Level& L = c.lv[l];
      if (L.fpending) {
        pend.push_back(std::move(L.fpend));
        L.fpend = FactorPending();
        L.fpending = false;
      } else {
        pend.push_back(factor_level_launch(c, L, c.stream));
      }
    }
    if (c.fwait) {
      CAV_HIP(hipStreamWaitEvent(c.stream, c.ev_fdone, 0));
      CAV_HIP(hipStreamWaitEvent(c.stream, c.ev_fdone2, 0));
      c.fwait = false;
    }
    for (int l = c.n_levels - 1, k = 0; l >= 1; --l, ++k) factor_level_finish(c, c.lv[l], pend[k], precision,
                                                                             cond_threshold, &st);
    if (c.coarse_pending) {
      c.coarse_pending = false;
      factor_coarse_finish(c, c.coarse_pend, c.side);
      c.coarse_ready = true;
      CAV_HIP(hipStreamWaitEvent(c.stream, c.ev_join, 0));
    }
  } catch (...) {
    (void)hipStreamSynchronize(c.stream);
    for (auto& fp : pend) factor_level_release(c, fp);
    throw;
  }
  st.coarse_cond_est = -1.0;
  if (out) *out = st;
  c.factored = true;
  return CAV_OK;
  API_END
}

cav_status cav_set_factor_layout(cav_ctx ctx, int layout) {
  if (!ctx) return CAV_ERR_INVALID_ARG;
  if (layout != CAV_LAYOUT_FULL && layout != CAV_LAYOUT_SYMMETRIC) {
    ctx->c.err = "unknown factor layout";
    return CAV_ERR_INVALID_ARG;
  }
  ctx->c.layout = layout;
  return CAV_OK;
}

cav_status cav_set_smoother(cav_ctx ctx, int kind, double alpha, int pre, int post) {
  if (!ctx) return CAV_ERR_INVALID_ARG;
  if (!std::isfinite(alpha) || pre < 0 || post < 0 || pre + post < 1 ||
      (kind != CAV_SMOOTHER_ADDITIVE && kind != CAV_SMOOTHER_MULTIPLICATIVE)) {
    ctx->c.err = "unknown smoother kind, or alpha not finite, or pre + post < 1";
    return CAV_ERR_INVALID_ARG;
  }
  ++ctx->c.generation;
  ctx->c.smoother = kind;
  ctx->c.alpha = alpha;
  ctx->c.pre = pre;
  ctx->c.post = post;
  return CAV_OK;
}

cav_status cav_apply_operator(cav_ctx ctx, const double* x, double* y) {
  if (!ctx) return CAV_ERR_INVALID_ARG;
  Ctx& c = ctx->c;
  API_BEGIN
  require(c.built, CAV_ERR_NOT_BUILT, "operator not built");
  require(x && y && x != y, CAV_ERR_INVALID_ARG, "x and y must be distinct device pointers");
  launch_apply_op(c.lv.back(), x, y, nullptr, c.stream);
  CAV_HIP(hipGetLastError());
  return CAV_OK;
  API_END
}

cav_status cav_vcycle(cav_ctx ctx, const double* r, double* z) {
  if (!ctx) return CAV_ERR_INVALID_ARG;
  Ctx& c = ctx->c;
  API_BEGIN
  require_factored(c, "cav_factor_patches has not succeeded");
  require(r && z && r != z, CAV_ERR_INVALID_ARG, "r and z must be distinct device pointers");
  vcycle_top(c, r, z);
  CAV_HIP(hipGetLastError());
  return CAV_OK;
  API_END
}

cav_status cav_fgmres_solve(cav_ctx ctx, const double* b, double* x, const cav_fgmres_opts* opts,
                            cav_solve_info* info) {
  if (!ctx) return CAV_ERR_INVALID_ARG;
  Ctx& c = ctx->c;
  API_BEGIN
  const int max_it = check_fgmres_args(c, b, x, opts);
  ensure_workspace(c, max_it);
  const KrylovWs ws{c.d_V, c.d_Z, c.d_w, c.d_bb, c.d_h, c.d_part, c.h_pinned};
  return fgmres_core(c, b, x, opts, info, ws);
  API_END
}

cav_status cav_fgmres_solve_noalloc(cav_ctx ctx, const double* b, double* x, const cav_fgmres_opts* opts,
                                    cav_solve_info* info) {
  if (!ctx) return CAV_ERR_INVALID_ARG;
  Ctx& c = ctx->c;
  API_BEGIN
  const int max_it = check_fgmres_args(c, b, x, opts);
  require(!(opts && opts->use_learned), CAV_ERR_INVALID_ARG,
          "cav_fgmres_solve_noalloc does not run the learned stage (its workspace is allocated on first use)");
  double* base = noalloc_scratch(c.device);
  require(base != nullptr, CAV_ERR_HIP, "the device address of the no-allocation scratch is not known");
  const int64_t n = 3 * int64_t(c.lv.back().N) * c.lv.back().N;
  const int64_t part = int64_t(dots_blocks(n)) * (max_it + 2);
  // blocks of the workspace, each starting on a 256-byte boundary (32 doubles)
  auto up = [](int64_t v) { return (v + 31) & ~int64_t(31); };
  const int64_t oV = 0, oZ = oV + up((max_it + 1) * n), ow = oZ + up(int64_t(max_it) * n), obb = ow + up(n),
                oh = obb + up(n), op = oh + up(3 * (max_it + 2)), total = op + up(part);
  if (total > int64_t(NOALLOC_SCRATCH_DOUBLES))
    throw StatusError(CAV_ERR_INVALID_ARG,
                      "cav_fgmres_solve_noalloc: max_it " + std::to_string(max_it) + " at " +
                          std::to_string(n) + " unknowns needs " + std::to_string(total * 8) +
                          " bytes of workspace; the fixed scratch holds " +
                          std::to_string(NOALLOC_SCRATCH_DOUBLES * 8) + " bytes");
  std::vector<double> hh(size_t(3 * (max_it + 2)));
  const KrylovWs ws{base + oV, base + oZ, base + ow, base + obb, base + oh, base + op, hh.data()};
  // no timing events either (creating one is a runtime allocation)
  const bool timing = c.timing;
  c.timing = false;
  try {
    const cav_status st = fgmres_core(c, b, x, opts, info, ws);
    c.timing = timing;
    return st;
  } catch (...) {
    c.timing = timing;
    throw;
  }
  API_END
}

int32_t cav_level_N(cav_ctx ctx, int level) {
  if (!ctx || level < 0 || level >= ctx->c.n_levels) return 0;
  return ctx->c.lv[level].N;
}

cav_status cav_level_apply(cav_ctx ctx, int level, int op, const double* x, double* y) {
  if (!ctx) return CAV_ERR_INVALID_ARG;
  Ctx& c = ctx->c;
  API_BEGIN
  require(c.built, CAV_ERR_NOT_BUILT, "operator not built");
  require(level >= 0 && level < c.n_levels, CAV_ERR_INVALID_ARG, "level out of range");
  require(x && y && x != y, CAV_ERR_INVALID_ARG, "x and y must be distinct device pointers");
  Level& L = c.lv[level];
  hipStream_t s = c.stream;
  switch (op) {
    case 0: launch_apply_op(L, x, y, nullptr, s); break;
    case 1:
      require(level >= 1, CAV_ERR_INVALID_ARG, "restriction needs level >= 1");
      launch_restrict(L, x, y, s);
      break;
    case 2: {
      require(level >= 1, CAV_ERR_INVALID_ARG, "prolongation needs level >= 1");
      const int64_t n = 3 * int64_t(L.N) * L.N;
      CAV_HIP(hipMemsetAsync(y, 0, size_t(n) * sizeof(double), s));
      launch_prolong_add(L, x, y, s);
      break;
    }
    case 3:
      require(level >= 1, CAV_ERR_NOT_BUILT, "smoother needs factored patches on level >= 1");
      require_factored(c, "smoother needs factored patches on level >= 1");
      launch_smoother(c, L, x, y, true, s);
      break;
    case 4:
      require(c.factored && level == 0, CAV_ERR_INVALID_ARG, "coarse solve is for level 0 after factorisation");
      launch_coarse_solve(c, x, y, s);
      break;
    case 5:
      require_factored(c, "V-cycle needs factored patches");
      vcycle_level(c, level, x, y);
      break;
    default: throw StatusError(CAV_ERR_INVALID_ARG, "unknown op");
  }
  CAV_HIP(hipGetLastError());
  return CAV_OK;
  API_END
}

cav_status cav_export_patches(cav_ctx ctx, int level, int64_t* offsets, int32_t* dofs, int64_t* total) {
  if (!ctx) return CAV_ERR_INVALID_ARG;
  Ctx& c = ctx->c;
  if (!c.patched || level < 1 || level >= c.n_levels) {
    c.err = "no patches on this level";
    return CAV_ERR_NOT_BUILT;
  }
  const Level& L = c.lv[level];
  if (total) *total = int64_t(L.patch_dofs.size());
  if (offsets) std::memcpy(offsets, L.patch_off.data(), L.patch_off.size() * sizeof(int64_t));
  if (dofs) std::memcpy(dofs, L.patch_dofs.data(), L.patch_dofs.size() * sizeof(int32_t));
  return CAV_OK;
}

cav_status cav_export_phases(cav_ctx ctx, int level, int32_t* ptr, int32_t* cells, int32_t* n_phases,
                             int32_t* n_cells) {
  if (!ctx) return CAV_ERR_INVALID_ARG;
  Ctx& c = ctx->c;
  if (!c.patched || level < 1 || level >= c.n_levels) {
    c.err = "no patches on this level";
    return CAV_ERR_NOT_BUILT;
  }
  Level& L = c.lv[level];
  API_BEGIN
  if (!L.coloured) colour_explicit(L.N, L.ee, L);
  if (n_phases) *n_phases = int32_t(L.ph_ptr.size()) - 1;
  if (n_cells) *n_cells = int32_t(L.ph_exp.size());
  if (ptr) std::memcpy(ptr, L.ph_ptr.data(), L.ph_ptr.size() * sizeof(int32_t));
  if (cells)
    for (size_t k = 0; k < L.ph_exp.size(); ++k) cells[k] = L.exp_cells[L.ph_exp[k]];
  return CAV_OK;
  API_END
}

cav_status cav_kernel_timing(cav_ctx ctx, int enable, cav_kernel_timing_info* out) {
  if (!ctx) return CAV_ERR_INVALID_ARG;
  Ctx& c = ctx->c;
  API_BEGIN
  if (out) {
    *out = cav_kernel_timing_info{};
    if (!c.kt_marks.empty() || !c.vc_marks.empty()) CAV_HIP(hipStreamSynchronize(c.stream));
    for (auto& m : c.kt_marks) {
      float ms = 0.f;
      CAV_HIP(hipEventElapsedTime(&ms, c.ev_pool[m.ev], c.ev_pool[m.ev + 1]));
      out->launches += m.launches;
      out->ms += ms;
      out->bytes += m.bytes;
      if (m.coop == 1 || m.coop == 2) {
        out->coop_launches += m.launches;
        out->coop_ms += ms;
        out->coop_bytes += m.bytes;
      }
      if (m.coop == 2) {
        out->shared_launches += m.launches;
        out->shared_ms += ms;
        out->shared_bytes += m.bytes;
      }
      if (m.coop == 3) {
        out->flow_launches += m.launches;
        out->flow_ms += ms;
        out->flow_bytes += m.bytes;
      }
    }
    for (auto& m : c.vc_marks) {
      float ms = 0.f;
      CAV_HIP(hipEventElapsedTime(&ms, c.ev_pool[m.first], c.ev_pool[m.second]));
      out->vcycles += 1;
      out->vcycle_ms += ms;
    }
  }
  c.kt_marks.clear();
  c.vc_marks.clear();
  c.ev_used = 0;
  c.timing = enable != 0;
  return CAV_OK;
  API_END
}

cav_status cav_export_ee(cav_ctx ctx, int level, int64_t* rowptr, int32_t* col, double* val, int64_t* nnz) {
  if (!ctx) return CAV_ERR_INVALID_ARG;
  Ctx& c = ctx->c;
  if (!c.built || level < 0 || level >= c.n_levels) {
    c.err = "operator not built or level out of range";
    return CAV_ERR_NOT_BUILT;
  }
  const HostCSR& E = c.lv[level].ee;
  if (nnz) *nnz = E.nnz();
  if (rowptr) std::memcpy(rowptr, E.rowptr.data(), E.rowptr.size() * sizeof(int64_t));
  if (col) std::memcpy(col, E.col.data(), E.col.size() * sizeof(int32_t));
  if (val) std::memcpy(val, E.val.data(), E.val.size() * sizeof(double));
  return CAV_OK;
}


cav_status cav_attach_net(cav_ctx ctx, cav_net net, double margin) {
  if (!ctx) return CAV_ERR_INVALID_ARG;
  Ctx& c = ctx->c;
  API_BEGIN
  require(std::isfinite(margin) && margin >= 0.0 && margin < 1.0, CAV_ERR_INVALID_ARG, "margin must be in [0, 1)");
  require(!net || net->n.device == c.device, CAV_ERR_INVALID_ARG, "net and context must share a device");
  c.net = net ? &net->n : nullptr;
  c.net_margin = margin;
  return CAV_OK;
  API_END
}

cav_status cav_learned_pairs(cav_ctx ctx, int32_t count, const double* xstar, int32_t iters, float* rhat,
                             float* ehat) {
  if (!ctx) return CAV_ERR_INVALID_ARG;
  Ctx& c = ctx->c;
  API_BEGIN
  require_factored(c, "cav_factor_patches has not succeeded");
  require(count >= 0 && iters >= 1 && iters <= 64, CAV_ERR_INVALID_ARG, "count >= 0 and 1 <= iters <= 64");
  if (count == 0) return CAV_OK;
  require(xstar && rhat && ehat, CAV_ERR_INVALID_ARG, "xstar, rhat and ehat must be device pointers");
  hipStream_t s = c.stream;
  Level& F = c.lv.back();
  const int64_t n = 3 * int64_t(F.N) * F.N;
  const int nbk = dots_blocks(n);
  // blocks of up to 16 solutions share each V-cycle (cav_vcycle_multi's cycle)
  const int64_t nb = int64_t(MR_COLS) * n;
  if (!c.d_pw || c.pw_n != n) {
    dev_free(c, c.d_pw);
    c.d_pw = static_cast<double*>(dev_alloc(c, size_t(5 * nb + MR_COLS + nbk) * sizeof(double)));
    c.pw_n = n;
  }
  ensure_multi_workspace(c);
  double* pb = c.d_pw;
  double* px = pb + nb;
  double* pr = pb + 2 * nb;
  double* pz = pb + 3 * nb;
  double* pe = pb + 4 * nb;
  double* nrm = pb + 5 * nb;
  double* part = nrm + MR_COLS;
  for (int32_t q0 = 0; q0 < count; q0 += MR_COLS) {
    const int kb = std::min<int32_t>(MR_COLS, count - q0);
    const double* xs = xstar + int64_t(q0) * n;
    for (int q = 0; q < kb; ++q) launch_apply_op(F, xs + q * n, pb + q * n, nullptr, s);  // b = K x*
    launch_fill(px, 0.0, kb * n, s);
    for (int32_t k = 0; k < iters; ++k) {
      for (int q = 0; q < kb; ++q) launch_apply_op(F, px + q * n, pr + q * n, pb + q * n, s);  // r = b - K x
      vcycle_level_multi(c, c.n_levels - 1, pr, pz, kb);
      k_axpby<<<nblocks(kb * n), TPB, 0, s>>>(px, 1.0, pz, 1.0, kb * n);
      k_axpby<<<nblocks(kb * n), TPB, 0, s>>>(pe, 1.0, xs, 0.0, kb * n);
      k_axpby<<<nblocks(kb * n), TPB, 0, s>>>(pe, -1.0, px, 1.0, kb * n);
      for (int q = 0; q < kb; ++q) {
        launch_apply_op(F, px + q * n, pr + q * n, pb + q * n, s);
        launch_dots(pr + q * n, n, 1, pr + q * n, n, part, nbk, nrm + q, s);
        const int64_t off = (int64_t(q0 + q) * iters + k) * n;
        launch_pair_write(pr + q * n, pe + q * n, nrm + q, rhat + off, ehat + off, n, s);
      }
    }
  }
  CAV_HIP(hipGetLastError());
  CAV_HIP(hipStreamSynchronize(s));
  return CAV_OK;
  API_END
}

cav_status cav_net_train_step_residual(cav_net net, cav_ctx ctx, int32_t kind, int32_t batch, const float* rhat,
                                       const int32_t* index, int64_t n_samples, double lr, double* loss) {
  if (!ctx) return CAV_ERR_INVALID_ARG;
  Ctx& c = ctx->c;
  API_BEGIN
  require(net != nullptr, CAV_ERR_INVALID_ARG, "net is NULL");
  require(c.built, CAV_ERR_NOT_BUILT, "operator not built");
  require(net->n.device == c.device, CAV_ERR_INVALID_ARG, "net and context must share a device");
  require(batch >= 1 && batch <= 65535, CAV_ERR_INVALID_ARG, "batch must be in [1, 65535]");
  require(rhat != nullptr, CAV_ERR_INVALID_ARG, "rhat must be a device pointer");
  require(std::isfinite(lr) && lr > 0.0, CAV_ERR_INVALID_ARG, "lr must be positive");
  require(kind == 0 || kind == 1, CAV_ERR_INVALID_ARG, "kind must be 0 (residual) or 1 (minimal residual)");
  Net& n = net->n;
  Level& F = c.lv.back();
  const int N = F.N;
  require(N >= 8, CAV_ERR_INVALID_ARG, "the finest grid must have N >= 8");
  hipStream_t s = c.stream;
  const int64_t n3 = 3 * int64_t(N) * N;
  const int32_t* didx = net_upload_index(n, index, batch, n_samples, s);
  net_forward_train(n, N, batch, rhat, didx, s);
  const int nbk = dots_blocks(n3);
  if (n.rl_n != n3) {
    if (n.d_rl) {
      net_dev_free(n, n.d_rl);
      n.d_rl = nullptr;
    }
    n.d_rl = static_cast<double*>(net_dev_alloc(n, size_t(4 * n3 + nbk) * sizeof(double)));
    n.rl_n = n3;
  }
  double* r64 = n.d_rl;
  double* c64 = r64 + n3;
  double* res = c64 + n3;
  double* q = res + n3;
  double* part = q + n3;
  double* sums = net_loss_sums(n, 3 * batch);  // 6 doubles per sample
  for (int b = 0; b < batch; ++b) {
    double* sb = sums + 6 * b;
    launch_sample_f64(rhat, didx, b, n3, r64, s);
    launch_sample_f64(n.d_y3, nullptr, b, n3, c64, s);
    if (kind == 0) {
      launch_apply_op(F, c64, res, r64, s);               // res = r - K c
      launch_dots(res, n3, 1, res, n3, part, nbk, sb, s);
      launch_dots(r64, n3, 1, r64, n3, part, nbk, sb + 1, s);
      launch_apply_op(F, res, q, nullptr, s);             // K^T (r - K c) = K (r - K c), K_E symmetric
      launch_scaled_f32(q, sb, -2.0 / batch, n3, n.d_g3 + b * n3, s);
    } else {
      launch_apply_op(F, c64, q, nullptr, s);             // q = K c
      launch_dots(q, n3, 1, r64, n3, part, nbk, sb, s);   // a = <Kc, r>
      launch_dots(q, n3, 1, q, n3, part, nbk, sb + 1, s); // b = ||Kc||^2
      launch_dots(r64, n3, 1, r64, n3, part, nbk, sb + 2, s);
      launch_mr_scalars(sb, batch, s);
      launch_sub_gamma(res, r64, q, sb, n3, s);           // res = r - gamma K c
      launch_apply_op(F, res, q, nullptr, s);             // K res
      launch_coef_f32(q, sb, n3, n.d_g3 + b * n3, s);     // -(2/B) a/(n b) K res
    }
  }
  net_backward_update(n, N, batch, rhat, didx, lr, s);
  std::vector<double> h(size_t(6) * batch);
  CAV_HIP(hipMemcpyAsync(h.data(), sums, h.size() * sizeof(double), hipMemcpyDeviceToHost, s));
  CAV_HIP(hipStreamSynchronize(s));
  if (loss) {
    double L = 0.0;
    for (int b = 0; b < batch; ++b) L += kind == 0 ? h[6 * b] / h[6 * b + 1] : h[6 * b + 4];
    *loss = L / batch;
  }
  return CAV_OK;
  API_END
}

cav_status cav_fgmres_solve_graph(cav_ctx ctx, const double* b, double* x, const cav_fgmres_opts* opts,
                                  cav_solve_info* info) {
  if (!ctx) return CAV_ERR_INVALID_ARG;
  Ctx& c = ctx->c;
  API_BEGIN
  require_factored(c, "cav_factor_patches has not succeeded");
  require(b && x && b != x, CAV_ERR_INVALID_ARG, "b and x must be distinct device pointers");
  require(!(opts && opts->use_learned), CAV_ERR_INVALID_ARG, "the graph solve has no learned stage");
  const double rtol = opts ? opts->rtol : 1e-10;
  const int max_it = opts ? opts->max_it : 150;
  require(max_it >= 1 && max_it <= 10000 && rtol >= 0.0, CAV_ERR_INVALID_ARG, "bad FGMRES options");
  return on_graph_stream(c, [&]() -> cav_status {
    graph_workspace(c, max_it);
    const Start st = graph_start(c, b);
    if (st.beta > 0.0) {
      if (!c.gexec || c.graph_generation != c.generation || c.graph_rtol != rtol) {
        drop_graph(c);
        c.gexec = capture_bodies({&c}, c.stream, rtol, &c.graph);
        c.graph_generation = c.generation;
        c.graph_rtol = rtol;
      }
      int32_t* done = reinterpret_cast<int32_t*>(c.h_pinned);
      for (int it = 0; it < max_it; ++it) {
        CAV_HIP(hipGraphLaunch(c.gexec, c.stream));
        CAV_HIP(hipMemcpyAsync(done, c.d_gi + GI_DONE, sizeof(int32_t), hipMemcpyDeviceToHost, c.stream));
        CAV_HIP(hipStreamSynchronize(c.stream));
        if (*done) break;
      }
    }
    return graph_finish(c, st, x, rtol, opts, info);
  });
  API_END
}

cav_status cav_batch_solve(cav_ctx* ctxs, int32_t n_sys, const double* const* b, double* const* x,
                           const cav_fgmres_opts* opts, cav_solve_info* infos, int32_t mode,
                           cav_batch_stats* stats) {
  if (!ctxs || n_sys < 1 || !b || !x) return CAV_ERR_INVALID_ARG;
  for (int i = 0; i < n_sys; ++i)
    if (!ctxs[i]) return CAV_ERR_INVALID_ARG;
  cav_ctx ctx = ctxs[0];
  Ctx& c0 = ctx->c;
  API_BEGIN
  require(mode == 0 || mode == 1, CAV_ERR_INVALID_ARG, "mode must be 0 (one graph) or 1 (graph per system)");
  require(!(opts && opts->use_learned), CAV_ERR_INVALID_ARG, "the batch solve has no learned stage");
  const double rtol = opts ? opts->rtol : 1e-10;
  const int max_it = opts ? opts->max_it : 150;
  require(max_it >= 1 && max_it <= 10000 && rtol >= 0.0, CAV_ERR_INVALID_ARG, "bad FGMRES options");
  for (int i = 0; i < n_sys; ++i) {
    Ctx& c = ctxs[i]->c;
    require_factored(c, "every context must be factored");
    require(c.device == c0.device, CAV_ERR_INVALID_ARG, "all contexts must share a device");
    require(b[i] && x[i] && b[i] != x[i], CAV_ERR_INVALID_ARG, "b and x must be distinct device pointers");
    for (int j = 0; j < i; ++j) require(ctxs[j] != ctxs[i], CAV_ERR_INVALID_ARG, "a context appears twice");
  }
  hipStream_t caller = c0.stream;
  hipStream_t origin = nullptr;
  CAV_HIP(hipStreamCreateWithFlags(&origin, hipStreamNonBlocking));
  hipEvent_t ev;
  CAV_HIP(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
  std::vector<hipStream_t> saved(n_sys, nullptr);
  std::vector<char> touched(n_sys, 0);
  std::vector<Start> starts(n_sys);
  std::vector<char> active(n_sys, 0);
  cav_batch_stats bs{};
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
  int32_t* flags = nullptr;
  cav_status ret = CAV_OK;
  struct Cleanup {
    std::function<void()> f;
    ~Cleanup() { f(); }
  } cleanup{[&]() {
    if (gexec) (void)hipGraphExecDestroy(gexec);
    if (graph) (void)hipGraphDestroy(graph);
    if (flags) (void)hipHostFree(flags);
    (void)hipStreamSynchronize(origin);
    for (int i = 0; i < n_sys; ++i)
      if (touched[i]) ctxs[i]->c.stream = saved[i];
    (void)hipEventRecord(ev, origin);
    (void)hipStreamWaitEvent(caller, ev, 0);
    (void)hipEventDestroy(ev);
    (void)hipStreamDestroy(origin);
  }};
  CAV_HIP(hipHostMalloc(reinterpret_cast<void**>(&flags), size_t(n_sys) * sizeof(int32_t), hipHostMallocDefault));
  CAV_HIP(hipEventRecord(ev, caller));
  CAV_HIP(hipStreamWaitEvent(origin, ev, 0));
  // prologues (each on its system's own stream)
  for (int i = 0; i < n_sys; ++i) {
    Ctx& c = ctxs[i]->c;
    graph_workspace(c, max_it);
    CAV_HIP(hipEventRecord(ev, c.stream));   // the system's caller-stream work comes first
    CAV_HIP(hipStreamWaitEvent(c.gstream, ev, 0));
    saved[i] = c.stream;
    touched[i] = 1;
    c.stream = c.gstream;
    starts[i] = graph_start(c, b[i]);
    active[i] = starts[i].beta > 0.0;
  }
  // rounds: one iteration of every active system per round
  std::vector<Ctx*> members;
  int launched_members = 0;
  for (int round = 0; round < max_it; ++round) {
    std::vector<Ctx*> act;
    std::vector<int> ids;
    for (int i = 0; i < n_sys; ++i)
      if (active[i]) {
        act.push_back(&ctxs[i]->c);
        ids.push_back(i);
      }
    if (act.empty()) break;
    if (mode == 0) {
      // recapture when a quarter of the graph's systems have finished
      if (!gexec || int(act.size()) * 4 <= launched_members * 3) {
        if (gexec) (void)hipGraphExecDestroy(gexec);
        if (graph) (void)hipGraphDestroy(graph);
        gexec = nullptr;
        graph = nullptr;
        // order each system's prior work before the origin stream
        for (Ctx* c : act) {
          hipEvent_t e;
          CAV_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
          CAV_HIP(hipEventRecord(e, c->stream));
          CAV_HIP(hipStreamWaitEvent(origin, e, 0));
          (void)hipEventDestroy(e);
        }
        gexec = capture_bodies(act, origin, rtol, &graph);
        launched_members = int(act.size());
        members = act;
        ++bs.captures;
      }
      CAV_HIP(hipGraphLaunch(gexec, origin));
      ++bs.graph_launches;
      for (int i = 0; i < n_sys; ++i)
        if (active[i])
          CAV_HIP(hipMemcpyAsync(flags + i, ctxs[i]->c.d_gi + GI_DONE, sizeof(int32_t), hipMemcpyDeviceToHost,
                                 origin));
      CAV_HIP(hipStreamSynchronize(origin));
    } else {
      for (size_t q = 0; q < act.size(); ++q) {
        Ctx& c = *act[q];
        if (!c.gexec || c.graph_generation != c.generation || c.graph_rtol != rtol) {
          drop_graph(c);
          c.gexec = capture_bodies({&c}, c.stream, rtol, &c.graph);
          c.graph_generation = c.generation;
          c.graph_rtol = rtol;
          ++bs.captures;
        }
        CAV_HIP(hipGraphLaunch(c.gexec, c.stream));
        ++bs.graph_launches;
        CAV_HIP(hipMemcpyAsync(flags + ids[q], c.d_gi + GI_DONE, sizeof(int32_t), hipMemcpyDeviceToHost, c.stream));
      }
      for (Ctx* c : act) CAV_HIP(hipStreamSynchronize(c->stream));
    }
    ++bs.rounds;
    for (int i : ids)
      if (flags[i]) active[i] = 0;
  }
  // the origin stream's graph work precedes each system's epilogue
  CAV_HIP(hipStreamSynchronize(origin));
  for (int i = 0; i < n_sys; ++i) {
    Ctx& c = ctxs[i]->c;
    cav_solve_info inf{};
    cav_status st = graph_finish(c, starts[i], x[i], rtol, nullptr, &inf);
    if (infos) infos[i] = inf;
    if (st != CAV_OK && ret == CAV_OK) ret = st;
    bs.iterations += inf.iterations;
  }
  if (stats) *stats = bs;
  return ret;
  API_END
}

cav_status cav_autotune(cav_ctx ctx, int32_t reps, int32_t* table) {
  if (!ctx) return CAV_ERR_INVALID_ARG;
  Ctx& c = ctx->c;
  API_BEGIN
  require_factored(c, "cav_factor_patches has not succeeded");
  require(reps >= 1 && reps <= 1000, CAV_ERR_INVALID_ARG, "reps must be in [1, 1000]");
  for (int l = 1; l < c.n_levels; ++l)
    require(!c.lv[l].packed, CAV_ERR_INVALID_ARG,
            "cav_autotune times the multiplicative phase kernels, which read full patch inverses");
  hipStream_t s = c.stream;
  hipEvent_t e0, e1;
  CAV_HIP(hipEventCreate(&e0));
  CAV_HIP(hipEventCreate(&e1));
  struct Ev {
    hipEvent_t a, b;
    ~Ev() {
      (void)hipEventDestroy(a);
      (void)hipEventDestroy(b);
    }
  } guard{e0, e1};
  const bool timing = c.timing;
  c.timing = false;
  launch_clear_sweep_flags(c, s);
  const int cand[7] = {256, 512, 1024, 0, 1, 2, 3};
  for (int l = 1; l < c.n_levels; ++l) {
    Level& L = c.lv[l];
    const int nph = int(L.ph_ptr.size()) - 1;
    if (nph <= 0) continue;
    const int64_t n = 3 * int64_t(L.N) * L.N;
    launch_fill(L.d_b, 1.0, n, s);
    launch_fill(L.d_x, 0.0, n, s);
    for (int bk = 0; bk < 4; ++bk) {
      std::vector<int> phs;
      for (int ph = 0; ph < nph; ++ph)
        if (mx_bucket(L.ph_maxn[ph]) == bk) phs.push_back(ph);
      if (phs.empty()) continue;
      float best = 1e30f;
      int pick = L.mx_nt[bk];
      for (int nt : cand) {
        for (int ph : phs) launch_mult_phase(c, L, ph, nt, L.d_b, L.d_x, s);  // warm-up
        CAV_HIP(hipEventRecord(e0, s));
        for (int r = 0; r < reps; ++r)
          for (int ph : phs) launch_mult_phase(c, L, ph, nt, L.d_b, L.d_x, s);
        CAV_HIP(hipEventRecord(e1, s));
        CAV_HIP(hipEventSynchronize(e1));
        CAV_HIP(hipGetLastError());
        float ms = 0.f;
        CAV_HIP(hipEventElapsedTime(&ms, e0, e1));
        if (ms < best) {
          best = ms;
          pick = nt;
        }
      }
      L.mx_nt[bk] = pick;
    }
    // The one-launch sweep (a cooperative launch) is not a candidate: it never
    // beat per-phase launches here, and a process's first cooperative launch
    // halves the concurrency of later graph launches on other streams. It
    // stays available through cav_set_tuning.
    L.sweep_mode = 0;
    // the dataflow sweep against the per-phase launches just chosen: the
    // whole explicit part of a sweep, `reps` times each
    if (L.flow_items > 0) {
      float t_mode[2] = {0.f, 0.f};
      for (int mode : {0, 2}) {
        L.sweep_mode = mode;
        launch_mult_smoother(c, L, L.d_b, L.d_x, false, s);   // warm-up
        CAV_HIP(hipEventRecord(e0, s));
        for (int r = 0; r < reps; ++r) launch_mult_smoother(c, L, L.d_b, L.d_x, false, s);
        CAV_HIP(hipEventRecord(e1, s));
        CAV_HIP(hipEventSynchronize(e1));
        CAV_HIP(hipGetLastError());
        CAV_HIP(hipEventElapsedTime(&t_mode[mode / 2], e0, e1));
      }
      L.sweep_mode = t_mode[1] < t_mode[0] ? 2 : 0;
    }
  }
  check_sweep_flags(c);
  c.timing = timing;
  ++c.generation;
  if (table)
    for (int l = 0; l < c.n_levels; ++l) {
      for (int bk = 0; bk < 4; ++bk) table[5 * l + bk] = c.lv[l].mx_nt[bk];
      table[5 * l + 4] = c.lv[l].sweep_mode;
    }
  return CAV_OK;
  API_END
}

cav_status cav_set_tuning(cav_ctx ctx, const int32_t* table) {
  if (!ctx) return CAV_ERR_INVALID_ARG;
  Ctx& c = ctx->c;
  API_BEGIN
  require(c.built && table != nullptr, CAV_ERR_INVALID_ARG, "needs a built context and a table");
  for (int l = 0; l < c.n_levels; ++l) {
    for (int bk = 0; bk < 4; ++bk) {
      const int v = table[5 * l + bk];
      require(v == 256 || v == 512 || v == 1024 || (v >= 0 && v <= 3), CAV_ERR_INVALID_ARG,
              "bucket entries must be 256, 512, 1024, 0 (split form), 1/2 (cooperative form, 64/128 rows) or 3 "
              "(cooperative form with a shared residual)");
    }
    require(table[5 * l + 4] >= 0 && table[5 * l + 4] <= 2, CAV_ERR_INVALID_ARG,
            "the sweep entry must be 0 (a launch per phase), 1 (one-launch sweep) or 2 (dataflow sweep)");
  }
  for (int l = 0; l < c.n_levels; ++l) {
    for (int bk = 0; bk < 4; ++bk) c.lv[l].mx_nt[bk] = table[5 * l + bk];
    c.lv[l].sweep_mode = table[5 * l + 4];
  }
  ++c.generation;
  return CAV_OK;
  API_END
}

cav_status cav_set_level_smoother(cav_ctx ctx, int level, int kind, double alpha) {
  if (!ctx) return CAV_ERR_INVALID_ARG;
  Ctx& c = ctx->c;
  API_BEGIN
  require(c.built, CAV_ERR_NOT_BUILT, "cav_build_operator has not succeeded");
  require(level >= 1 && level < c.n_levels, CAV_ERR_INVALID_ARG, "level must be a smoothed level (1 .. n_levels-1)");
  require(kind == -1 || kind == CAV_SMOOTHER_ADDITIVE || kind == CAV_SMOOTHER_MULTIPLICATIVE, CAV_ERR_INVALID_ARG,
          "kind must be -1 or a CAV_SMOOTHER_* value");
  require(kind == -1 || std::isfinite(alpha), CAV_ERR_INVALID_ARG, "alpha must be finite");
  c.lv[level].smoother = kind;
  c.lv[level].alpha = alpha;
  ++c.generation;
  return CAV_OK;
  API_END
}

cav_status cav_vcycle_multi(cav_ctx ctx, int32_t k, const double* R, double* Z) {
  if (!ctx) return CAV_ERR_INVALID_ARG;
  Ctx& c = ctx->c;
  API_BEGIN
  require_factored(c, "cav_factor_patches has not succeeded");
  require(k >= 0, CAV_ERR_INVALID_ARG, "k must be non-negative");
  if (k == 0) return CAV_OK;
  require(R && Z && R != Z, CAV_ERR_INVALID_ARG, "R and Z must be distinct device pointers");
  ensure_multi_workspace(c);
  const int64_t n = 3 * int64_t(c.lv.back().N) * c.lv.back().N;
  for (int32_t q0 = 0; q0 < k; q0 += MR_COLS)
    vcycle_level_multi(c, c.n_levels - 1, R + q0 * n, Z + q0 * n, std::min<int32_t>(MR_COLS, k - q0));
  CAV_HIP(hipGetLastError());
  return CAV_OK;
  API_END
}

cav_status cav_error_propagation(cav_ctx ctx, int32_t k, const double* X, double* T) {
  if (!ctx) return CAV_ERR_INVALID_ARG;
  Ctx& c = ctx->c;
  API_BEGIN
  require_factored(c, "cav_factor_patches has not succeeded");
  require(k >= 0, CAV_ERR_INVALID_ARG, "k must be non-negative");
  if (k == 0) return CAV_OK;
  require(X && T && X != T, CAV_ERR_INVALID_ARG, "X and T must be distinct device pointers");
  ensure_multi_workspace(c);
  Level& F = c.lv.back();
  hipStream_t s = c.stream;
  const int64_t n = 3 * int64_t(F.N) * F.N;
  // the finest level's block buffer holds K x (the cycle uses it only below the finest level)
  for (int32_t q0 = 0; q0 < k; q0 += MR_COLS) {
    const int kb = std::min<int32_t>(MR_COLS, k - q0);
    for (int q = 0; q < kb; ++q) launch_apply_op(F, X + (q0 + q) * n, F.d_mb + q * n, nullptr, s);  // w = K x
    vcycle_level_multi(c, c.n_levels - 1, F.d_mb, T + q0 * n, kb);                              // t = V(K x)
    k_axpby<<<nblocks(kb * n), TPB, 0, s>>>(T + q0 * n, 1.0, X + q0 * n, -1.0, kb * n);         // t = x - V(K x)
  }
  CAV_HIP(hipGetLastError());
  return CAV_OK;
  API_END
}

cav_status cav_set_phase_order(cav_ctx ctx, int order) {
  if (!ctx) return CAV_ERR_INVALID_ARG;
  Ctx& c = ctx->c;
  if (order != CAV_ORDER_EXPLICIT_FIRST && order != CAV_ORDER_STANDARD_FIRST) {
    c.err = "order must be CAV_ORDER_EXPLICIT_FIRST or CAV_ORDER_STANDARD_FIRST";
    return CAV_ERR_INVALID_ARG;
  }
  c.std_first = order == CAV_ORDER_STANDARD_FIRST;
  ++c.generation;
  return CAV_OK;
}

cav_status cav_set_wait_limit(cav_ctx ctx, uint32_t polls) {
  if (!ctx) return CAV_ERR_INVALID_ARG;
  ctx->c.wait_limit = polls;
  return CAV_OK;
}

}  // extern "C"

cav_status cav_ib_interpolate(cav_ctx ctx, const double* x, double* U) {
  if (!ctx) return CAV_ERR_INVALID_ARG;
  Ctx& c = ctx->c;
  API_BEGIN
  require(c.built, CAV_ERR_NOT_BUILT, "operator not built");
  build_ib_tables(c);
  if (c.ib_rows == 0) return CAV_OK;
  require(x && U, CAV_ERR_INVALID_ARG, "x and U must be device pointers");
  k_ib_interp<<<nblocks(c.ib_rows), TPB, 0, c.stream>>>(c.ib_rows, c.d_ib_face, c.d_ib_w, x, U);
  CAV_HIP(hipGetLastError());
  return CAV_OK;
  API_END
}

cav_status cav_ib_spread_add(cav_ctx ctx, const double* F, double* y) {
  if (!ctx) return CAV_ERR_INVALID_ARG;
  Ctx& c = ctx->c;
  API_BEGIN
  require(c.built, CAV_ERR_NOT_BUILT, "operator not built");
  build_ib_tables(c);
  if (c.ib_faces == 0) return CAV_OK;
  require(F && y, CAV_ERR_INVALID_ARG, "F and y must be device pointers");
  k_ib_spread<<<nblocks(c.ib_faces), TPB, 0, c.stream>>>(c.ib_faces, c.d_sp_face, c.d_sp_ptr, c.d_sp_row, c.d_sp_w, F,
                                                          y);
  CAV_HIP(hipGetLastError());
  return CAV_OK;
  API_END
}

cav_status cav_structure_force(const cav_structure_desc* st, double* F) {
  if (!st || !F) return CAV_ERR_INVALID_ARG;
  try {
    std::vector<double> f;
    std::string err;
    const cav_status s = fibre_force(st, f, err);
    if (s != CAV_OK) return s;
    std::copy(f.begin(), f.end(), F);
    return CAV_OK;
  } catch (const std::bad_alloc&) {
    return CAV_ERR_OUT_OF_MEMORY;
  }
}

cav_status cav_newton_solve(cav_ctx ctx, const cav_grid_desc* g, const cav_structure_desc* st, const double* rhs,
                            double* x, double* X_new, const cav_newton_opts* o, cav_newton_info* info) {
  if (!ctx) return CAV_ERR_INVALID_ARG;
  Ctx& c = ctx->c;
  std::vector<void*> bufs;
  auto release = [&]() {
    for (void* p : bufs) dev_free(c, p);
    bufs.clear();
  };
  cav_newton_info inf{};
  std::vector<double> Xk;
  bool have_X = false;
  // every exit reports what was reached: counts, residuals, the last configuration
  auto report = [&]() {
    if (info) *info = inf;
    if (X_new && have_X) std::copy(Xk.begin(), Xk.end(), X_new);
  };
  int stage = 0;
  try {
    require(g && st && o && rhs && x && rhs != x, CAV_ERR_INVALID_ARG,
            "grid, structure, options, rhs and x are required (rhs and x distinct)");
    require(st->law == CAV_LAW_FIBRE, CAV_ERR_INVALID_ARG, "the Newton step needs the fibre law");
    require(std::isfinite(o->rtol) && o->rtol >= 0 && std::isfinite(o->atol) && o->atol >= 0 && o->max_newton >= 0 &&
                o->max_newton <= 1000 && std::isfinite(o->lin_rtol) && o->lin_rtol >= 0 && o->lin_max_it >= 1,
            CAV_ERR_INVALID_ARG, "bad Newton options");
    auto call = [&](cav_status s) {
      if (s != CAV_OK) throw StatusError(s, c.err);
    };
    stage = 1;
    cav_structure_desc d = *st;
    d.X_force = nullptr;
    d.X_disp = nullptr;
    // J^n, S^n and the Stokes stencil at X^n (the operator itself is rebuilt per correction)
    call(cav_build_operator(ctx, g, &d));
    const int M = st->M;
    const int64_t n2 = int64_t(g->N) * g->N, n = 3 * n2;
    const StencilCoef sc = c.lv.back().sc;
    auto alloc = [&](size_t bytes) {
      void* p = dev_alloc(c, bytes);
      bufs.push_back(p);
      return p;
    };
    double* dU = static_cast<double*>(alloc(2 * size_t(M) * sizeof(double)));
    double* dF = static_cast<double*>(alloc(2 * size_t(M) * sizeof(double)));
    double* dy = static_cast<double*>(alloc(size_t(n) * sizeof(double)));
    double* ddx = static_cast<double*>(alloc(size_t(n) * sizeof(double)));
    const int nblk = dots_blocks(n);
    double* dpart = static_cast<double*>(alloc(size_t(nblk) * sizeof(double)));
    double* dnrm = static_cast<double*>(alloc(sizeof(double)));
    Xk.assign(2 * size_t(M), 0.0);
    std::vector<double> U(2 * size_t(M)), disp(2 * size_t(M)), Fh;
    const std::vector<double> Xn(st->X, st->X + 2 * size_t(M));
    std::vector<double> built(2 * size_t(M), 0.0);  // displacement of the operator the context holds
    cav_fgmres_opts fo{};
    fo.rtol = o->lin_rtol;
    fo.max_it = o->lin_max_it;
    hipStream_t s = c.stream;
    for (int it = 0;; ++it) {
      // X_k = X^n + dt J^n u_k and the force there
      stage = 5;
      if (M > 0) {
        call(cav_ib_interpolate(ctx, x, dU));
        CAV_HIP(hipMemcpyAsync(U.data(), dU, U.size() * sizeof(double), hipMemcpyDeviceToHost, s));
        CAV_HIP(hipStreamSynchronize(s));
      }
      // the energies see X^n displaced by dt J^n u_k, links updated incrementally
      for (size_t k = 0; k < Xk.size(); ++k) {
        disp[k] = g->dt * U[k];
        Xk[k] = Xn[k] + disp[k];
      }
      have_X = true;
      d.X_disp = disp.data();
      std::string err;
      const cav_status fs = fibre_force(&d, Fh, err);
      if (fs != CAV_OK) throw StatusError(fs, err);
      if (M > 0) CAV_HIP(hipMemcpyAsync(dF, Fh.data(), Fh.size() * sizeof(double), hipMemcpyHostToDevice, s));
      // y = rhs + S^n F(X_k) - K_0 x = -R(x)
      launch_stencil(sc, x, dy, rhs, s);
      call(cav_ib_spread_add(ctx, dF, dy));
      launch_dots(dy, n, 1, dy, n, dpart, nblk, dnrm, s);
      double r2 = 0.0;
      CAV_HIP(hipMemcpyAsync(&r2, dnrm, sizeof(double), hipMemcpyDeviceToHost, s));
      CAV_HIP(hipStreamSynchronize(s));
      const double rn = std::sqrt(r2);
      require(std::isfinite(rn), CAV_ERR_INVALID_ARG, "non-finite Newton residual");
      if (it == 0) inf.res0 = rn;
      inf.res = rn;
      if (rn <= o->rtol * inf.res0 || rn <= o->atol) {
        inf.converged = 1;
        break;
      }
      if (it == o->max_newton) break;
      // the Newton system at X_k: hierarchy rebuilt with E = DF[X_k] (the
      // operator is kept when X_k is the configuration it was built at, as for
      // the first correction from rest)
      if (disp != built) {
        stage = 1;
        call(cav_build_operator(ctx, g, &d));
        built = disp;
      }
      stage = 2;
      call(cav_build_cav_patches(ctx, o->family, nullptr));
      stage = 3;
      call(cav_factor_patches(ctx, o->precision, o->cond_threshold, nullptr));
      call(cav_set_smoother(ctx, o->smoother, o->alpha, 1, 1));
      stage = 4;
      cav_solve_info si{};
      const cav_status ls = cav_fgmres_solve(ctx, dy, ddx, &fo, &si);
      if (ls == CAV_WARN_NOT_CONVERGED)
        ++inf.lin_unconverged;  // the correction is FGMRES's best: inexact Newton
      else if (ls != CAV_OK && ls != CAV_WARN_FLOOR_LIMITED)
        throw StatusError(ls, c.err);
      k_axpby<<<nblocks(n), TPB, 0, s>>>(x, 1.0, ddx, 1.0, n);
      CAV_HIP(hipGetLastError());
      ++inf.newton_its;
      inf.fgmres_its_total += si.iterations;
      inf.fgmres_its_max = std::max(inf.fgmres_its_max, si.iterations);
    }
    CAV_HIP(hipStreamSynchronize(s));
    release();
    report();
    return inf.converged ? CAV_OK : CAV_WARN_NOT_CONVERGED;
  } catch (const StatusError& e) {
    c.err = e.msg;
    release();
    inf.failed_stage = stage;
    report();
    return e.st;
  } catch (const HipError& e) {
    c.err = e.msg;
    release();
    inf.failed_stage = stage;
    report();
    return CAV_ERR_HIP;
  } catch (const std::bad_alloc&) {
    c.err = "host allocation failed";
    release();
    inf.failed_stage = stage;
    report();
    return CAV_ERR_OUT_OF_MEMORY;
  }
}
