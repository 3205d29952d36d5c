// Host-only analysis handle: the setup that precedes any device work (force
// law, E_E = S E J, Galerkin coarsening, patch families, colour phases),
// exported for inspection and for checks on machines without a GPU.
#include <cmath>
#include <cstring>
#include <new>

#include "cav_internal.hpp"

struct cav_analysis_s {
  std::vector<cav::Level> lv;
  int n_levels = 0;
  bool patched = false;
};

extern "C" {

static cav_status analyze(const cav_grid_desc* g, const cav_structure_desc* st, int family, int box_b, int box_o,
                          cav_analysis* out) {
  if (!g || !out) return CAV_ERR_INVALID_ARG;
  const int N = g->N, L = g->n_levels;
  if (!(N >= 4 && (N & (N - 1)) == 0) || L < 1 || L > 30 || (N >> (L - 1)) < 4) return CAV_ERR_INVALID_ARG;
  if (family != CAV_FAMILY_CAV && family != CAV_FAMILY_VANKA && family != CAV_FAMILY_BOX) return CAV_ERR_INVALID_ARG;
  if (family == CAV_FAMILY_BOX) {
    if (box_b < 1 || box_o < 0) return CAV_ERR_INVALID_ARG;
    for (int l = 1; l < L; ++l)
      if ((N >> (L - 1 - l)) % box_b != 0) return CAV_ERR_INVALID_ARG;
  }
  cav::Structure S;
  std::string err;
  const cav_status ss = cav::make_structure(st, S, err);
  if (ss != CAV_OK) return ss;
  cav_analysis a = new (std::nothrow) cav_analysis_s();
  if (!a) return CAV_ERR_OUT_OF_MEMORY;
  try {
    a->n_levels = L;
    a->lv.resize(L);
    for (int l = 0; l < L; ++l) a->lv[l].N = N >> (L - 1 - l);
    cav::assemble_ee_finest(N, S, a->lv[L - 1].ee);
    for (int l = L - 1; l >= 1; --l) cav::galerkin_coarsen(a->lv[l - 1].N, a->lv[l].ee, a->lv[l - 1].ee);
    for (int l = 1; l < L; ++l) {
      if (family == CAV_FAMILY_BOX)
        cav::build_box_patches(a->lv[l].N, a->lv[l].ee, box_b, box_o, a->lv[l]);
      else
        cav::build_patches(a->lv[l].N, a->lv[l].ee, family, a->lv[l]);
    }
    a->patched = true;
  } catch (const std::bad_alloc&) {
    delete a;
    return CAV_ERR_OUT_OF_MEMORY;
  }
  *out = a;
  return CAV_OK;
}

cav_status cav_analyze(const cav_grid_desc* g, const cav_structure_desc* st, int family, cav_analysis* out) {
  if (family == CAV_FAMILY_BOX) return CAV_ERR_INVALID_ARG;
  return analyze(g, st, family, 0, 0, out);
}

cav_status cav_analyze_box(const cav_grid_desc* g, const cav_structure_desc* st, int b, int o, cav_analysis* out) {
  return analyze(g, st, CAV_FAMILY_BOX, b, o, out);
}

cav_status cav_analysis_destroy(cav_analysis a) {
  delete a;
  return CAV_OK;
}

cav_status cav_analysis_export_ee(cav_analysis a, int level, int64_t* rowptr, int32_t* col, double* val,
                                  int64_t* nnz) {
  if (!a || level < 0 || level >= a->n_levels) return CAV_ERR_INVALID_ARG;
  const cav::HostCSR& E = a->lv[level].ee;
  if (nnz) *nnz = E.nnz();
  if (rowptr) std::memcpy(rowptr, E.rowptr.data(), E.rowptr.size() * sizeof(int64_t));
  if (col) std::memcpy(col, E.col.data(), E.col.size() * sizeof(int32_t));
  if (val) std::memcpy(val, E.val.data(), E.val.size() * sizeof(double));
  return CAV_OK;
}

cav_status cav_analysis_export_patches(cav_analysis a, int level, int64_t* offsets, int32_t* dofs, int64_t* total) {
  if (!a || level < 1 || level >= a->n_levels) return CAV_ERR_INVALID_ARG;
  const cav::Level& L = a->lv[level];
  if (total) *total = int64_t(L.patch_dofs.size());
  if (offsets) std::memcpy(offsets, L.patch_off.data(), L.patch_off.size() * sizeof(int64_t));
  if (dofs) std::memcpy(dofs, L.patch_dofs.data(), L.patch_dofs.size() * sizeof(int32_t));
  return CAV_OK;
}

cav_status cav_analysis_export_phases(cav_analysis a, int level, int32_t* ptr, int32_t* cells, int32_t* n_phases,
                                      int32_t* n_cells) {
  if (!a || level < 1 || level >= a->n_levels) return CAV_ERR_INVALID_ARG;
  const cav::Level& L = a->lv[level];
  if (n_phases) *n_phases = int32_t(L.ph_ptr.size()) - 1;
  if (n_cells) *n_cells = int32_t(L.ph_exp.size());
  if (ptr) std::memcpy(ptr, L.ph_ptr.data(), L.ph_ptr.size() * sizeof(int32_t));
  if (cells)
    for (size_t k = 0; k < L.ph_exp.size(); ++k) cells[k] = L.exp_cells[L.ph_exp[k]];
  return CAV_OK;
}

cav_status cav_analysis_export_weights(cav_analysis a, int level, int32_t* dofs, double* inv_cnt,
                                       int32_t* n_touched) {
  if (!a || level < 1 || level >= a->n_levels) return CAV_ERR_INVALID_ARG;
  const cav::Level& L = a->lv[level];
  if (n_touched) *n_touched = L.n_touched;
  if (dofs) std::memcpy(dofs, L.t_dof_h.data(), L.t_dof_h.size() * sizeof(int32_t));
  if (inv_cnt) std::memcpy(inv_cnt, L.t_inv_h.data(), L.t_inv_h.size() * sizeof(double));
  return CAV_OK;
}

}  // extern "C"
