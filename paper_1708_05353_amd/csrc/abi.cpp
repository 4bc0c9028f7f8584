// extern "C" entry points of libocck: argument validation, error reporting,
// handle lifetime.  Host only; the GPU work lives in far_k.hip.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <new>
#include <stdexcept>
#include <unordered_set>

#include "occk_internal.hpp"

namespace occk {

static thread_local std::string g_err = "";

void set_error(const std::string& msg) { g_err = msg; }

static std::mutex g_mu;
static std::unordered_set<const Tree*> g_live;

static bool live(const Tree* t) {
  std::lock_guard<std::mutex> lk(g_mu);
  return t && g_live.count(t) && t->magic == kTreeMagic;
}

static std::unordered_set<const void*> g_plans;
static std::unordered_set<const void*> g_sels;

static bool sel_live(const void* p) {
  std::lock_guard<std::mutex> lk(g_mu);
  return p && g_sels.count(p) && selector_live(p);
}

static bool plan_live(const void* p) {
  std::lock_guard<std::mutex> lk(g_mu);
  return p && g_plans.count(p);
}

}  // namespace occk

using namespace occk;

#define OCCK_GUARD_BEGIN try {
#define OCCK_GUARD_END                                             \
  }                                                                \
  catch (const std::invalid_argument& e) {                        \
    set_error(e.what());                                           \
    return OCCK_EINVAL;                                            \
  }                                                                \
  catch (const std::bad_alloc&) {                                  \
    set_error("host allocation failed");                           \
    return OCCK_ENOMEM;                                            \
  }                                                                \
  catch (const std::exception& e) {                                \
    set_error(e.what());                                           \
    return OCCK_EINVAL;                                            \
  }                                                                \
  catch (...) {                                                    \
    set_error("unknown error");                                    \
    return OCCK_EINVAL;                                            \
  }

extern "C" {

int32_t occk_abi_version(void) { return OCCK_ABI_VERSION; }

const char* occk_last_error(void) { return g_err.c_str(); }

int32_t occk_build_tree(const occk_system* sys, const occk_tree_params* params, occk_tree** out) {
  if (!out) {
    set_error("out is NULL");
    return OCCK_EINVAL;
  }
  *out = nullptr;
  OCCK_GUARD_BEGIN
  Tree* t = build_tree(sys, params);
  {
    std::lock_guard<std::mutex> lk(g_mu);
    g_live.insert(t);
  }
  *out = reinterpret_cast<occk_tree*>(t);
  return OCCK_OK;
  OCCK_GUARD_END
}

int32_t occk_free_tree(occk_tree* tree) {
  if (!tree) return OCCK_OK;
  Tree* t = reinterpret_cast<Tree*>(tree);
  {
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_live.count(t) || t->magic != kTreeMagic) {
      set_error("occk_free_tree: handle is not live");
      return OCCK_EHANDLE;
    }
    g_live.erase(t);
  }
  device_free(t);
  jstate_free(t);
  nstate_free(t);
  t->magic = 0;
  delete t;
  return OCCK_OK;
}

int32_t occk_tree_info(const occk_tree* tree, occk_tree_info_t* info) {
  const Tree* t = reinterpret_cast<const Tree*>(tree);
  if (!live(t)) {
    set_error("occk_tree_info: handle is not live");
    return OCCK_EHANDLE;
  }
  if (!info) {
    set_error("info is NULL");
    return OCCK_EINVAL;
  }
  std::memset(info, 0, sizeof(*info));
  const int D = t->params.depth;
  info->nbasis = t->nbasis;
  info->lmax = t->L;
  info->ncomp = t->Q;
  info->depth = D;
  info->lmin = t->lmin;
  info->nleaf = t->nleaf();
  for (int lev = 0; lev <= D && lev < OCCK_MAX_LEVELS; ++lev) {
    info->boxes_per_level[lev] = int32_t(t->boxes[lev].size());
    info->il_per_level[lev] = int32_t(t->il_idx[lev].size());
    info->n_il += int64_t(t->il_idx[lev].size());
    if (t->lmin >= 0 && lev >= t->lmin) info->nbox += int32_t(t->boxes[lev].size());
    if (t->lmin >= 0 && lev > t->lmin) info->n_edges += int64_t(t->boxes[lev].size());
  }
  info->npairs = int64_t(t->pairs.size());
  for (const auto& f : t->leaf_funcs) {
    info->sum_nb += int64_t(f.size());
    info->sum_nb2 += int64_t(f.size()) * int64_t(f.size());
    info->max_nb = std::max<int32_t>(info->max_nb, int32_t(f.size()));
  }
  info->n_ops = int32_t(t->ops.size());
  info->m2m_nnz = t->m2m_nnz;
  for (int d = 0; d < 3; ++d) {
    info->lo[d] = t->lo[d];
    info->mid[d] = t->mid[d];
  }
  info->width = t->W;
  info->n_near = int64_t(t->near_idx.size());
  return OCCK_OK;
}

int32_t occk_tree_near(const occk_tree* tree, int32_t* ptr, int32_t* idx) {
  const Tree* t = reinterpret_cast<const Tree*>(tree);
  if (!live(t)) {
    set_error("occk_tree_near: handle is not live");
    return OCCK_EHANDLE;
  }
  if (ptr) std::copy(t->near_ptr.begin(), t->near_ptr.end(), ptr);
  if (idx) std::copy(t->near_idx.begin(), t->near_idx.end(), idx);
  return OCCK_OK;
}

int32_t occk_tree_flops(const occk_tree* tree, int32_t ni, int32_t nj, int32_t symmetric, occk_flops_t* out) {
  const Tree* t = reinterpret_cast<const Tree*>(tree);
  if (!live(t)) {
    set_error("occk_tree_flops: handle is not live");
    return OCCK_EHANDLE;
  }
  if (!out || ni < 0 || nj < 0 || (symmetric && ni != nj)) {
    set_error("occk_tree_flops: out must be non-NULL, ni, nj >= 0, and ni == nj when symmetric");
    return OCCK_EINVAL;
  }
  std::memset(out, 0, sizeof(*out));
  if (t->lmin < 0) return OCCK_OK;
  const int D = t->params.depth;
  int64_t n_il = 0, n_edges = 0, sum_nb = 0;
  for (int lev = 0; lev <= D; ++lev) {
    n_il += int64_t(t->il_idx[lev].size());
    if (lev > t->lmin) n_edges += int64_t(t->boxes[lev].size());
  }
  for (const auto& f : t->leaf_funcs) sum_nb += int64_t(f.size());
  const int64_t Q = t->Q, a = ni, b = nj;
  const int64_t nc = symmetric ? a * (a + 1) / 2 : a * b;
  out->half = 2 * Q * b * int64_t(t->pairs.size());
  out->omega = symmetric ? Q * a * (a + 1) * sum_nb : 2 * Q * a * b * sum_nb;
  out->m2m = 2 * t->m2m_nnz * nc * n_edges;
  out->m2l = 2 * Q * Q * nc * n_il;
  out->l2l = out->m2m;
  out->l2p = 2 * Q * a * b * sum_nb;
  out->total = out->half + out->omega + out->m2m + out->m2l + out->l2l + out->l2p;
  return OCCK_OK;
}

int32_t occk_tree_export(const occk_tree* tree, int32_t* leaf_coords, int32_t* il_level,
                         int32_t* il_target, int32_t* il_source, int32_t* pair_leaf) {
  const Tree* t = reinterpret_cast<const Tree*>(tree);
  if (!live(t)) {
    set_error("occk_tree_export: handle is not live");
    return OCCK_EHANDLE;
  }
  const int D = t->params.depth;
  if (leaf_coords)
    for (size_t b = 0; b < t->boxes[D].size(); ++b)
      for (int d = 0; d < 3; ++d) leaf_coords[3 * b + d] = t->boxes[D][b][d];
  int64_t k = 0;
  for (int lev = 0; lev <= D; ++lev) {
    const auto& bx = t->boxes[lev];
    for (size_t b = 0; b < bx.size(); ++b)
      for (int32_t e = t->il_ptr[lev][b]; e < t->il_ptr[lev][b + 1]; ++e, ++k) {
        const auto& c2 = bx[t->il_idx[lev][e]];
        if (il_level) il_level[k] = lev;
        if (il_target) il_target[k] = int32_t(coord_key(bx[b][0], bx[b][1], bx[b][2]));
        if (il_source) il_source[k] = int32_t(coord_key(c2[0], c2[1], c2[2]));
      }
  }
  if (pair_leaf)
    for (size_t p = 0; p < t->pairs.size(); ++p) pair_leaf[p] = t->pairs[p].leaf;
  return OCCK_OK;
}

int32_t occk_tree_leaf(const occk_tree* tree, int32_t leaf, int32_t* nb, int32_t* funcs, double* O) {
  const Tree* t = reinterpret_cast<const Tree*>(tree);
  if (!live(t)) {
    set_error("occk_tree_leaf: handle is not live");
    return OCCK_EHANDLE;
  }
  if (leaf < 0 || leaf >= t->nleaf()) {
    set_error("leaf index out of range");
    return OCCK_EINVAL;
  }
  OCCK_GUARD_BEGIN
  const auto& f = t->leaf_funcs[leaf];
  if (nb) *nb = int32_t(f.size());
  if (funcs) std::copy(f.begin(), f.end(), funcs);
  if (O) leaf_multipoles(*t, leaf, O);
  return OCCK_OK;
  OCCK_GUARD_END
}

}  // extern "C"

// Host-side checks shared by occk_far_K and occk_far_K_noalloc; fills o.
static int32_t check_far_K(const char* fn, Tree* t, const double* C, int64_t ldc, int32_t nocc, int32_t i0,
                           int32_t i1, int32_t j0, int32_t j1, const occk_far_opts* opts, double* K, int64_t ldk,
                           occk_far_opts& o) {
  const std::string f(fn);
  if (!live(t)) {
    set_error(f + ": handle is not live");
    return OCCK_EHANDLE;
  }
  if (!C || !K) {
    set_error(f + ": C and K must be non-NULL device pointers");
    return OCCK_EINVAL;
  }
  if (nocc <= 0 || ldc < nocc) {
    set_error(f + ": need nocc > 0 and ldc >= nocc");
    return OCCK_EINVAL;
  }
  if (!(0 <= i0 && i0 <= i1 && i1 <= nocc) || !(0 <= j0 && j0 <= j1 && j1 <= nocc)) {
    set_error(f + ": need 0 <= i0 <= i1 <= nocc and 0 <= j0 <= j1 <= nocc");
    return OCCK_EINVAL;
  }
  if (ldk < i1 || ldk <= 0) {
    set_error(f + ": need ldk >= i1");
    return OCCK_EINVAL;
  }
  if ((reinterpret_cast<uintptr_t>(C) | reinterpret_cast<uintptr_t>(K)) & 7) {
    set_error(f + ": C and K must be 8-byte aligned");
    return OCCK_EINVAL;
  }
  {
    const uintptr_t c0 = reinterpret_cast<uintptr_t>(C);
    const uintptr_t c1 = c0 + uintptr_t(t->nbasis) * uintptr_t(ldc) * 8;
    const uintptr_t k0 = reinterpret_cast<uintptr_t>(K);
    const uintptr_t k1 = k0 + uintptr_t(t->nbasis) * uintptr_t(ldk) * 8;
    if (c0 < k1 && k0 < c1) {
      set_error(f + ": K overlaps C");
      return OCCK_EINVAL;
    }
  }
  if (t->L > kMaxL) {
    set_error(f + ": the exchange kernels take lmax <= 8 (the tree has a higher rank, for occk_far_J)");
    return OCCK_EINVAL;
  }
  o = occk_far_opts{};
  if (opts) o = *opts;
  if (o.precision < OCCK_PREC_FP64 || o.precision > OCCK_PREC_BF16X6) {
    set_error(f + ": unknown precision");
    return OCCK_EINVAL;
  }
  if (o.rank_mode != OCCK_RANK_FIXED && o.rank_mode != OCCK_RANK_LEARNED) {
    set_error(f + ": unknown rank_mode");
    return OCCK_EINVAL;
  }
  if (o.rank_mode == OCCK_RANK_LEARNED && !sel_live(o.selector)) {
    set_error(f + ": LEARNED rank mode needs a live selector");
    return OCCK_ESTATE;
  }
  if (o.jblock < 0) {
    set_error(f + ": jblock must be >= 0");
    return OCCK_EINVAL;
  }
  if (o.lds_tree != 0 && o.lds_tree != 1) {
    set_error(f + ": lds_tree must be 0 or 1");
    return OCCK_EINVAL;
  }
  if (o.one_stream != 0 && o.one_stream != 1) {
    set_error(f + ": one_stream must be 0 or 1");
    return OCCK_EINVAL;
  }
  if (!(o.pair_thresh >= 0.0) || !std::isfinite(o.pair_thresh) ||
      (o.pair_thresh > 0.0 && (i0 != j0 || i1 != j1))) {
    set_error(f + ": pair_thresh must be finite and >= 0, and screening needs i0 == j0 and i1 == j1");
    return OCCK_EINVAL;
  }
  return OCCK_OK;
}

extern "C" {

int32_t occk_far_K(occk_tree* tree, const double* C, int64_t ldc, int32_t nocc, int32_t i0, int32_t i1,
                   int32_t j0, int32_t j1, const occk_far_opts* opts, double* K, int64_t ldk,
                   void* hip_stream) {
  Tree* t = reinterpret_cast<Tree*>(tree);
  occk_far_opts o{};
  const int32_t rc = check_far_K("occk_far_K", t, C, ldc, nocc, i0, i1, j0, j1, opts, K, ldk, o);
  if (rc != OCCK_OK) return rc;
  OCCK_GUARD_BEGIN
  return far_K(t, C, ldc, nocc, i0, i1, j0, j1, &o, K, ldk, hip_stream);
  OCCK_GUARD_END
}

int32_t occk_far_K_noalloc(occk_tree* tree, const double* C, int64_t ldc, int32_t nocc, int32_t i0, int32_t i1,
                           int32_t j0, int32_t j1, const occk_far_opts* opts, double* K, int64_t ldk,
                           void* hip_stream) {
  Tree* t = reinterpret_cast<Tree*>(tree);
  occk_far_opts o{};
  const int32_t rc = check_far_K("occk_far_K_noalloc", t, C, ldc, nocc, i0, i1, j0, j1, opts, K, ldk, o);
  if (rc != OCCK_OK) return rc;
  if (o.precision != OCCK_PREC_FP64 || o.rank_mode != OCCK_RANK_FIXED || o.pair_thresh != 0.0) {
    set_error("occk_far_K_noalloc: only FP64 with fixed rank and no pair screening");
    return OCCK_EINVAL;
  }
  OCCK_GUARD_BEGIN
  return far_K_noalloc(t, C, ldc, nocc, i0, i1, j0, j1, &o, K, ldk, hip_stream);
  OCCK_GUARD_END
}

int32_t occk_far_J(occk_tree* tree, const double* D, int64_t ldd, double* J, int64_t ldj, int32_t accumulate,
                   void* hip_stream) {
  Tree* t = reinterpret_cast<Tree*>(tree);
  if (!live(t)) {
    set_error("occk_far_J: handle is not live");
    return OCCK_EHANDLE;
  }
  const int64_t n = t->nbasis;
  if (!D || !J || ldd < n || ldj < n || (accumulate != 0 && accumulate != 1)) {
    set_error("occk_far_J: D and J must be non-NULL, ldd and ldj >= nbasis, accumulate 0 or 1");
    return OCCK_EINVAL;
  }
  if ((reinterpret_cast<uintptr_t>(D) | reinterpret_cast<uintptr_t>(J)) & 7) {
    set_error("occk_far_J: D and J must be 8-byte aligned");
    return OCCK_EINVAL;
  }
  {
    const uintptr_t d0 = reinterpret_cast<uintptr_t>(D), d1 = d0 + uintptr_t(n) * uintptr_t(ldd) * 8;
    const uintptr_t j0 = reinterpret_cast<uintptr_t>(J), j1 = j0 + uintptr_t(n) * uintptr_t(ldj) * 8;
    if (d0 < j1 && j0 < d1) {
      set_error("occk_far_J: J overlaps D");
      return OCCK_EINVAL;
    }
  }
  OCCK_GUARD_BEGIN
  return far_J(t, D, ldd, J, ldj, accumulate, hip_stream);
  OCCK_GUARD_END
}

int32_t occk_near_K(occk_tree* tree, const double* C, int64_t ldc, int32_t nocc, double* K, int64_t ldk,
                    int32_t accumulate, void* hip_stream) {
  Tree* t = reinterpret_cast<Tree*>(tree);
  if (!live(t)) {
    set_error("occk_near_K: handle is not live");
    return OCCK_EHANDLE;
  }
  if (!C || !K || nocc <= 0 || ldc < nocc || ldk < nocc || (accumulate != 0 && accumulate != 1)) {
    set_error("occk_near_K: C and K non-NULL, nocc > 0, ldc and ldk >= nocc, accumulate 0 or 1");
    return OCCK_EINVAL;
  }
  if ((reinterpret_cast<uintptr_t>(C) | reinterpret_cast<uintptr_t>(K)) & 7) {
    set_error("occk_near_K: C and K must be 8-byte aligned");
    return OCCK_EINVAL;
  }
  {
    const uintptr_t c0 = reinterpret_cast<uintptr_t>(C), c1 = c0 + uintptr_t(t->nbasis) * uintptr_t(ldc) * 8;
    const uintptr_t k0 = reinterpret_cast<uintptr_t>(K), k1 = k0 + uintptr_t(t->nbasis) * uintptr_t(ldk) * 8;
    if (c0 < k1 && k0 < c1) {
      set_error("occk_near_K: K overlaps C");
      return OCCK_EINVAL;
    }
  }
  OCCK_GUARD_BEGIN
  return near_K(t, C, ldc, nocc, K, ldk, accumulate, hip_stream);
  OCCK_GUARD_END
}

int32_t occk_pair_screen_info(occk_tree* tree, int64_t* carried, int32_t* jblock, int32_t* band_end, int32_t cap,
                              int32_t* nband) {
  Tree* t = reinterpret_cast<Tree*>(tree);
  if (!live(t)) {
    set_error("occk_pair_screen_info: handle is not live");
    return OCCK_EHANDLE;
  }
  if (!carried || !jblock || !nband || cap < 0 || (cap > 0 && !band_end)) {
    set_error("occk_pair_screen_info: NULL pointer or negative cap");
    return OCCK_EINVAL;
  }
  return pair_screen_info(t, carried, jblock, band_end, cap, nband);
}

int32_t occk_near_info(occk_tree* tree, int64_t* tasks, int64_t* quartets) {
  Tree* t = reinterpret_cast<Tree*>(tree);
  if (!live(t)) {
    set_error("occk_near_info: handle is not live");
    return OCCK_EHANDLE;
  }
  const int32_t rc = near_K_counts(t, tasks, quartets);
  if (rc != OCCK_OK) set_error("occk_near_info: no occk_near_K call on this handle yet");
  return rc;
}

int32_t occk_tree_flops_J(const occk_tree* tree, occk_jflops_t* out) {
  const Tree* t = reinterpret_cast<const Tree*>(tree);
  if (!live(t)) {
    set_error("occk_tree_flops_J: handle is not live");
    return OCCK_EHANDLE;
  }
  if (!out) {
    set_error("occk_tree_flops_J: out is NULL");
    return OCCK_EINVAL;
  }
  std::memset(out, 0, sizeof(*out));
  if (t->lmin < 0) return OCCK_OK;
  const int D = t->params.depth;
  int64_t n_il = 0, n_edges = 0;
  for (int lev = 0; lev <= D; ++lev) {
    n_il += int64_t(t->il_idx[lev].size());
    if (lev > t->lmin) n_edges += int64_t(t->boxes[lev].size());
  }
  const int64_t Q = t->Q, np = int64_t(t->pairs.size());
  out->dens = 2 * Q * np;
  out->m2m = 2 * t->m2m_nnz * n_edges;
  out->m2l = 2 * Q * Q * n_il;
  out->l2l = out->m2m;
  out->pair = 2 * Q * np;
  out->total = out->dens + out->m2m + out->m2l + out->l2l + out->pair;
  return OCCK_OK;
}

int32_t occk_debug_mfma_probe(int32_t kind, int32_t ia, int32_t ka, int32_t jb, double* host_out) {
  const int kmax = kind == 2 ? 31 : 3;
  if (!host_out || kind < 0 || kind > 2 || ia < 0 || ia > 15 || jb < 0 || jb > 15 || ka < 0 || ka > kmax) {
    set_error("occk_debug_mfma_probe: bad arguments");
    return OCCK_EINVAL;
  }
  return debug_mfma_probe(kind, ia, ka, jb, host_out);
}

int32_t occk_debug_buffer(occk_tree* tree, int32_t which, double* host, int64_t* count) {
  Tree* t = reinterpret_cast<Tree*>(tree);
  if (!live(t)) {
    set_error("occk_debug_buffer: handle is not live");
    return OCCK_EHANDLE;
  }
  if (which < 0 || which > 3) {
    set_error("occk_debug_buffer: which must be 0..3");
    return OCCK_EINVAL;
  }
  return debug_buffer(t, which, host, count);
}

int32_t occk_profile_enable(occk_tree* tree, int32_t enable) {
  Tree* t = reinterpret_cast<Tree*>(tree);
  if (!live(t)) {
    set_error("occk_profile_enable: handle is not live");
    return OCCK_EHANDLE;
  }
  t->profile = enable ? 1 : 0;
  return OCCK_OK;
}

int32_t occk_profile_read(occk_tree* tree, double* ms, int64_t* launches) {
  Tree* t = reinterpret_cast<Tree*>(tree);
  if (!live(t)) {
    set_error("occk_profile_read: handle is not live");
    return OCCK_EHANDLE;
  }
  return profile_read(t, ms, launches);
}

int32_t occk_workspace_info(occk_tree* tree, int32_t* jblock, int64_t* bytes) {
  Tree* t = reinterpret_cast<Tree*>(tree);
  if (!live(t)) {
    set_error("occk_workspace_info: handle is not live");
    return OCCK_EHANDLE;
  }
  return workspace_info(t, jblock, bytes);
}

int32_t occk_batch_create(int32_t nsys, occk_tree* const* trees, const int32_t* nocc, const occk_far_opts* opts,
                          occk_batch** out) {
  if (!out) {
    set_error("occk_batch_create: out is NULL");
    return OCCK_EINVAL;
  }
  *out = nullptr;
  if (nsys < 1 || nsys > 4096 || !trees || !nocc) {
    set_error("occk_batch_create: need 1 <= nsys <= 4096 and non-NULL trees, nocc");
    return OCCK_EINVAL;
  }
  occk_far_opts o{};
  if (opts) o = *opts;
  if (o.precision < OCCK_PREC_FP64 || o.precision > OCCK_PREC_BF16X6) {
    set_error("occk_batch_create: unknown precision");
    return OCCK_EINVAL;
  }
  if (o.rank_mode != OCCK_RANK_FIXED || o.pair_thresh != 0.0) {
    set_error("occk_batch_create: only fixed ranks without pair screening are batched");
    return OCCK_EINVAL;
  }
  if (o.jblock < 0) {
    set_error("occk_batch_create: jblock must be >= 0");
    return OCCK_EINVAL;
  }
  std::vector<Tree*> ts(nsys);
  for (int k = 0; k < nsys; ++k) {
    Tree* t = reinterpret_cast<Tree*>(trees[k]);
    if (!live(t)) {
      set_error("occk_batch_create: a tree handle is not live");
      return OCCK_EHANDLE;
    }
    for (int k2 = 0; k2 < k; ++k2)
      if (ts[k2] == t) {
        set_error("occk_batch_create: a tree appears twice");
        return OCCK_EINVAL;
      }
    if (t->lmin < 0) {
      set_error("occk_batch_create: a system has no far field");
      return OCCK_EINVAL;
    }
    if (t->L > kMaxL) {
      set_error("occk_batch_create: the exchange kernels take lmax <= 8");
      return OCCK_EINVAL;
    }
    if (t->L != reinterpret_cast<Tree*>(trees[0])->L) {
      set_error("occk_batch_create: all systems must share lmax");
      return OCCK_EINVAL;
    }
    if (nocc[k] < 1) {
      set_error("occk_batch_create: nocc must be >= 1");
      return OCCK_EINVAL;
    }
    ts[k] = t;
  }
  void* plan = nullptr;
  int32_t rc = OCCK_OK;
  OCCK_GUARD_BEGIN
  rc = batch_create(nsys, ts.data(), nocc, o.precision, o.jblock, &plan);
  OCCK_GUARD_END
  if (rc != OCCK_OK) return rc;
  {
    std::lock_guard<std::mutex> lk(g_mu);
    g_plans.insert(plan);
  }
  *out = reinterpret_cast<occk_batch*>(plan);
  return OCCK_OK;
}

int32_t occk_batch_shape(const occk_batch* plan, int32_t* nsys, int32_t* nocc, int32_t cap) {
  if (!plan_live(plan)) {
    set_error("occk_batch_shape: plan is not live");
    return OCCK_EHANDLE;
  }
  return batch_shape(plan, nsys, nocc, cap, nullptr);
}

int32_t occk_batch_config(const occk_batch* plan, int32_t* config) {
  if (!plan_live(plan)) {
    set_error("occk_batch_config: plan is not live");
    return OCCK_EHANDLE;
  }
  if (!config) {
    set_error("occk_batch_config: config is NULL");
    return OCCK_EINVAL;
  }
  return batch_shape(plan, nullptr, nullptr, 0, config);
}

int32_t occk_batch_stage_times(occk_batch* plan, double* ms, int32_t* type, int32_t cap, int32_t* nstage) {
  if (!plan_live(plan)) {
    set_error("occk_batch_stage_times: plan is not live");
    return OCCK_EHANDLE;
  }
  if (cap < 0 || (cap > 0 && !ms && !type)) {
    set_error("occk_batch_stage_times: cap must be >= 0, with ms or type non-NULL when cap > 0");
    return OCCK_EINVAL;
  }
  return batch_stage_times(plan, ms, type, cap, nstage);
}

static int32_t check_io(int nsys, const double* const* C, const int64_t* ldc, double* const* K, const int64_t* ldk) {
  if (!C || !ldc || !K || !ldk) {
    set_error("batch: NULL array argument");
    return OCCK_EINVAL;
  }
  for (int k = 0; k < nsys; ++k)
    if (!C[k] || !K[k] || ((reinterpret_cast<uintptr_t>(C[k]) | reinterpret_cast<uintptr_t>(K[k])) & 7)) {
      set_error("batch: C and K pointers must be non-NULL and 8-byte aligned");
      return OCCK_EINVAL;
    }
  return OCCK_OK;
}

int32_t occk_batch_run(occk_batch* plan, const double* const* C, const int64_t* ldc, double* const* K,
                       const int64_t* ldk, void* hip_stream) {
  if (!plan_live(plan)) {
    set_error("occk_batch_run: plan is not live");
    return OCCK_EHANDLE;
  }
  int32_t nsys = 0;
  int32_t rc = occk_batch_shape(plan, &nsys, nullptr, 0);
  if (rc != OCCK_OK) return rc;
  if ((rc = check_io(nsys, C, ldc, K, ldk)) != OCCK_OK) return rc;
  std::vector<int32_t> nocc(nsys);
  occk_batch_shape(plan, &nsys, nocc.data(), nsys);
  for (int k = 0; k < nsys; ++k)
    if (ldc[k] < nocc[k] || ldk[k] < nocc[k]) {
      set_error("occk_batch_run: need ldc >= nocc and ldk >= nocc");
      return OCCK_EINVAL;
    }
  OCCK_GUARD_BEGIN
  return batch_run(plan, C, ldc, K, ldk, hip_stream);
  OCCK_GUARD_END
}

int32_t occk_batch_tune(occk_batch* plan, const double* const* C, const int64_t* ldc, double* const* K,
                        const int64_t* ldk, void* hip_stream, int32_t* choice) {
  if (!plan_live(plan)) {
    set_error("occk_batch_tune: plan is not live");
    return OCCK_EHANDLE;
  }
  int32_t nsys = 0;
  occk_batch_shape(plan, &nsys, nullptr, 0);
  int32_t rc = check_io(nsys, C, ldc, K, ldk);
  if (rc != OCCK_OK) return rc;
  OCCK_GUARD_BEGIN
  return batch_tune(plan, C, ldc, K, ldk, hip_stream, choice);
  OCCK_GUARD_END
}

int32_t occk_batch_free(occk_batch* plan) {
  if (!plan) return OCCK_OK;
  {
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_plans.count(plan)) {
      set_error("occk_batch_free: plan is not live");
      return OCCK_EHANDLE;
    }
    g_plans.erase(plan);
  }
  return batch_free(plan);
}

int32_t occk_far_K_batched(int32_t nsys, occk_tree* const* trees, const double* const* C, const int64_t* ldc,
                           const int32_t* nocc, const occk_far_opts* opts, double* const* K, const int64_t* ldk,
                           void* hip_stream) {
  if (nsys >= 1 && nsys <= 4096 && trees && nocc) {   // the I/O arrays are checked before any plan is made
    const int32_t rc = check_io(nsys, C, ldc, K, ldk);
    if (rc != OCCK_OK) return rc;
  }
  occk_batch* plan = nullptr;
  int32_t rc = occk_batch_create(nsys, trees, nocc, opts, &plan);
  if (rc != OCCK_OK) return rc;
  rc = occk_batch_run(plan, C, ldc, K, ldk, hip_stream);
  std::string msg = rc != OCCK_OK ? occk_last_error() : "";
  const int32_t rf = occk_batch_free(plan);   // synchronises the device: the launch has finished
  if (rc != OCCK_OK) {
    set_error(msg);
    return rc;
  }
  return rf;
}

int32_t occk_selector_create(int32_t seed, occk_selector** out) {
  if (!out) {
    set_error("occk_selector_create: out is NULL");
    return OCCK_EINVAL;
  }
  *out = nullptr;
  void* p = nullptr;
  int32_t rc = OCCK_OK;
  OCCK_GUARD_BEGIN
  rc = selector_create(seed, &p);
  OCCK_GUARD_END
  if (rc != OCCK_OK) return rc;
  {
    std::lock_guard<std::mutex> lk(g_mu);
    g_sels.insert(p);
  }
  *out = reinterpret_cast<occk_selector*>(p);
  return OCCK_OK;
}

int32_t occk_selector_free(occk_selector* sel) {
  if (!sel) return OCCK_OK;
  {
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_sels.count(sel)) {
      set_error("occk_selector_free: selector is not live");
      return OCCK_EHANDLE;
    }
    g_sels.erase(sel);
  }
  return selector_free(sel);
}

#define OCCK_SEL_CHECK(s)                          \
  if (!sel_live(s)) {                              \
    set_error("selector handle is not live");      \
    return OCCK_EHANDLE;                           \
  }

int32_t occk_selector_get_weights(const occk_selector* sel, float* theta) {
  OCCK_SEL_CHECK(sel)
  if (!theta) {
    set_error("theta is NULL");
    return OCCK_EINVAL;
  }
  return selector_weights(const_cast<occk_selector*>(sel), theta, nullptr);
}

int32_t occk_selector_set_weights(occk_selector* sel, const float* theta) {
  OCCK_SEL_CHECK(sel)
  if (!theta) {
    set_error("theta is NULL");
    return OCCK_EINVAL;
  }
  for (int k = 0; k < OCCK_SELECTOR_NPARAM; ++k)
    if (!std::isfinite(theta[k])) {
      set_error("occk_selector_set_weights: non-finite weight");
      return OCCK_ENONFINITE;
    }
  return selector_weights(sel, nullptr, theta);
}

int32_t occk_selector_set_rule(occk_selector* sel, float log10_tau, float margin) {
  OCCK_SEL_CHECK(sel)
  if (!std::isfinite(log10_tau) || !std::isfinite(margin)) {
    set_error("occk_selector_set_rule: non-finite rule");
    return OCCK_ENONFINITE;
  }
  selector_set_rule(sel, log10_tau, margin);
  return OCCK_OK;
}

static int32_t check_samples(const float* X, const float* T, int32_t n, int nt) {
  if (!X || (nt && !T) || n < 1) {
    set_error("need n >= 1 and non-NULL sample arrays");
    return OCCK_EINVAL;
  }
  for (int64_t k = 0; k < int64_t(n) * OCCK_SELECTOR_NFEAT; ++k)
    if (!std::isfinite(X[k])) {
      set_error("non-finite feature");
      return OCCK_ENONFINITE;
    }
  for (int64_t k = 0; k < int64_t(n) * nt; ++k)
    if (!std::isfinite(T[k])) {
      set_error("non-finite target");
      return OCCK_ENONFINITE;
    }
  return OCCK_OK;
}

int32_t occk_selector_train(occk_selector* sel, const float* feat, const float* target, int32_t n, int32_t epochs,
                            int32_t batch, float lr, int32_t seed, float* loss, void* hip_stream) {
  OCCK_SEL_CHECK(sel)
  int32_t rc = check_samples(feat, target, n, OCCK_SELECTOR_NOUT);
  if (rc != OCCK_OK) return rc;
  if (epochs < 1 || batch < 1 || !(lr > 0.f) || !std::isfinite(lr)) {
    set_error("occk_selector_train: need epochs >= 1, batch >= 1, lr > 0");
    return OCCK_EINVAL;
  }
  OCCK_GUARD_BEGIN
  return selector_train(sel, feat, target, n, epochs, batch, lr, seed, loss, hip_stream);
  OCCK_GUARD_END
}

int32_t occk_selector_grad(occk_selector* sel, const float* feat, const float* target, int32_t n, float* loss,
                           float* grad, void* hip_stream) {
  OCCK_SEL_CHECK(sel)
  int32_t rc = check_samples(feat, target, n, OCCK_SELECTOR_NOUT);
  if (rc != OCCK_OK) return rc;
  if (!grad) {
    set_error("grad is NULL");
    return OCCK_EINVAL;
  }
  OCCK_GUARD_BEGIN
  return selector_grad(sel, feat, target, n, loss, grad, hip_stream);
  OCCK_GUARD_END
}

int32_t occk_selector_predict(occk_selector* sel, const float* feat, int32_t n, int32_t lmax, float* out,
                              int32_t* rank, void* hip_stream) {
  OCCK_SEL_CHECK(sel)
  int32_t rc = check_samples(feat, nullptr, n, 0);
  if (rc != OCCK_OK) return rc;
  if (lmax < 1 || lmax > 8) {
    set_error("occk_selector_predict: lmax must be in [1, 8]");
    return OCCK_EINVAL;
  }
  OCCK_GUARD_BEGIN
  return selector_predict(sel, feat, n, lmax, out, rank, hip_stream);
  OCCK_GUARD_END
}

int32_t occk_selector_save(const occk_selector* sel, const char* path) {
  OCCK_SEL_CHECK(sel)
  if (!path) {
    set_error("path is NULL");
    return OCCK_EINVAL;
  }
  return selector_save(sel, path);
}

int32_t occk_selector_load(occk_selector* sel, const char* path) {
  OCCK_SEL_CHECK(sel)
  if (!path) {
    set_error("path is NULL");
    return OCCK_EINVAL;
  }
  return selector_load(sel, path);
}

int32_t occk_selector_collect(occk_tree* tree, const double* C, int64_t ldc, int32_t nocc, int32_t j0, int32_t j1,
                              int32_t max_samples, int32_t seed, float* feat, float* target, int32_t* nsamples,
                              void* hip_stream) {
  Tree* t = reinterpret_cast<Tree*>(tree);
  if (!live(t)) {
    set_error("occk_selector_collect: handle is not live");
    return OCCK_EHANDLE;
  }
  if (!C || !feat || !target || !nsamples || max_samples < 1 || nocc < 1 || ldc < nocc ||
      !(0 <= j0 && j0 < j1 && j1 <= nocc)) {
    set_error("occk_selector_collect: bad arguments");
    return OCCK_EINVAL;
  }
  if (t->lmin < 0 || t->L > kMaxL) {
    set_error("occk_selector_collect: the tree has no far field or a rank above 8");
    return OCCK_EINVAL;
  }
  OCCK_GUARD_BEGIN
  return selector_collect(t, C, ldc, nocc, j0, j1, max_samples, seed, feat, target, nsamples, hip_stream);
  OCCK_GUARD_END
}

int32_t occk_rank_stats(occk_tree* tree, int64_t* hist) {
  Tree* t = reinterpret_cast<Tree*>(tree);
  if (!live(t)) {
    set_error("occk_rank_stats: handle is not live");
    return OCCK_EHANDLE;
  }
  if (!hist) {
    set_error("hist is NULL");
    return OCCK_EINVAL;
  }
  return rank_stats(t, hist);
}

}  // extern "C"
