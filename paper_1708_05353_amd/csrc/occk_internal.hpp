// Internal state of the occk library (not part of the ABI).
#pragma once

#include <cstdint>
#include <string>
#include <unordered_map>
#include <vector>

#include "../../include/occk.h"

namespace occk {

constexpr uint32_t kTreeMagic = 0x6f63636bu;  // "occk"
constexpr int kMaxL = 8;        // multipole rank of the exchange kernels
constexpr int kMaxLTree = 15;   // multipole rank of a tree (the Coulomb path takes up to 15)

void set_error(const std::string& msg);

struct Func {
  double c[3];
  double exp;
  double norm;
  int pw[3];   // Cartesian powers (0/1)
  int32_t shell;
};

// One screened ordered AO function pair.
struct Pair {
  int32_t r, s;
  double P[3];
  int32_t leaf;
};

// Translation operator description; the matrix itself is generated on the GPU.
enum OpType : int32_t { kOpM2M = 0, kOpL2L = 1, kOpM2L = 2 };
struct OpDesc {
  int32_t type;
  int32_t weighted;   // rows scaled by the L2P weights (leaf-level L2L/M2L)
  double d[3];        // displacement: Xc - Xp (M2M/L2L) or X - X' (M2L)
};

struct DeviceState;   // defined in the HIP translation unit
struct JState;        // device state of the Coulomb path (far_j.hip)
struct NState;        // device state of the near-field exchange (near_k.hip)

struct Tree {
  uint32_t magic = kTreeMagic;
  occk_tree_params params{};
  int L = 0, Q = 0, nbasis = 0, ndim = 0;
  std::vector<Func> funcs;
  std::vector<Pair> pairs;
  double lo[3]{}, mid[3]{}, W = 0;
  int lmin = -1;
  // boxes[level] = sorted integer coordinates (x, y, z)
  std::vector<std::vector<std::array<int32_t, 3>>> boxes;
  std::vector<std::unordered_map<int64_t, int32_t>> index;
  // interaction lists per level: CSR over the boxes of that level
  std::vector<std::vector<int32_t>> il_ptr, il_idx;
  // leaves near each leaf (itself included): the near field, CSR over the leaves
  std::vector<int32_t> near_ptr, near_idx;
  std::vector<int32_t> shell_first, shell_l;   // first function and l of every shell
  // leaves
  std::vector<std::vector<int32_t>> leaf_funcs;   // sorted function indices
  std::vector<std::vector<int32_t>> leaf_pairs;   // indices into pairs
  // operators
  std::vector<OpDesc> ops;
  std::vector<int32_t> op_up;     // [level][octant] -> op (M2M), -1 if unused
  std::vector<int32_t> op_down;   // [level][octant] -> op (L2L)
  // M2L op per (level, displacement key)
  std::vector<std::unordered_map<int64_t, int32_t>> op_m2l;
  int64_t m2m_nnz = 0;

  DeviceState* dev = nullptr;
  JState* jdev = nullptr;     // device state of the Coulomb path (far_j.hip)
  NState* ndev = nullptr;     // device state of the near-field path (near_k.hip)
  int profile = 0;

  double h(int level) const { return W / double(int64_t(1) << level); }
  int nsplit() const { return ndim; }
  void centre(int level, const std::array<int32_t, 3>& c, double out[3]) const;
  int32_t parent(int level, int32_t box) const;
  int nleaf() const { return int(boxes.back().size()); }
};

inline int64_t coord_key(int32_t x, int32_t y, int32_t z) {
  return int64_t(x) + 4096 * (int64_t(y) + 4096 * int64_t(z));
}

// Real form: component (l,0) -> l*l, Re(l,m) -> l*l+2m-1, Im(l,m) -> l*l+2m.
inline int rq0(int l) { return l * l; }
inline int rqre(int l, int m) { return l * l + 2 * m - 1; }
inline int rqim(int l, int m) { return l * l + 2 * m; }

// Dense real-form AO multipole block of one leaf (Q x nb x nb), FP64, host.
void leaf_multipoles(const Tree& t, int leaf, double* out);
// Real-form AO multipoles of the leaf's pairs, [pair][q] in leaf_pairs order, FP64, host.
void leaf_pair_multipoles(const Tree& t, int leaf, double* out);

// Builds everything host-side; throws std::runtime_error / std::bad_alloc.
Tree* build_tree(const occk_system* sys, const occk_tree_params* p);

// Device side (far_k.hip)
void device_free(Tree* t);
int32_t far_K(Tree* t, const double* C, int64_t ldc, int32_t nocc, int32_t i0, int32_t i1,
              int32_t j0, int32_t j1, const occk_far_opts* opts, double* K, int64_t ldk,
              void* stream);
int32_t far_K_noalloc(Tree* t, const double* C, int64_t ldc, int32_t nocc, int32_t i0, int32_t i1,
                      int32_t j0, int32_t j1, const occk_far_opts* opts, double* K, int64_t ldk, void* stream);
void jstate_free(Tree* t);
void nstate_free(Tree* t);
int32_t near_K(Tree* t, const double* C, int64_t ldc, int32_t nocc, double* K, int64_t ldk, int32_t accumulate,
               void* stream);
int32_t near_K_counts(Tree* t, int64_t* tasks, int64_t* quartets);
int32_t far_J(Tree* t, const double* D, int64_t ldd, double* J, int64_t ldj, int32_t accumulate, void* stream);
int32_t debug_mfma_probe(int kind, int ia, int ka, int jb, double* host_out);
int32_t debug_buffer(Tree* t, int which, double* host, int64_t* count);
int32_t profile_read(Tree* t, double* ms, int64_t* launches);
int32_t workspace_info(Tree* t, int32_t* jblock, int64_t* bytes);
int32_t pair_screen_info(Tree* t, int64_t* carried, int32_t* jblock, int32_t* band_end, int32_t cap, int32_t* nband);
int32_t batch_create(int nsys, Tree* const* trees, const int32_t* nocc, int prec, int jblock, void** out);
int32_t batch_run(void* plan, const double* const* C, const int64_t* ldc, double* const* K, const int64_t* ldk,
                  void* stream);
int32_t batch_tune(void* plan, const double* const* C, const int64_t* ldc, double* const* K, const int64_t* ldk,
                   void* stream, int32_t* choice);
int32_t batch_free(void* plan);
int32_t batch_stage_times(void* plan, double* ms, int32_t* type, int cap, int32_t* nstage);
int32_t batch_shape(const void* plan, int32_t* nsys, int32_t* nocc, int cap, int32_t* tuned);
int32_t selector_create(int32_t seed, void** out);
int32_t selector_free(void* sel);
int32_t selector_weights(void* sel, float* get, const float* set);
void selector_set_rule(void* sel, float log10_tau, float margin);
int32_t selector_train(void* sel, const float* X, const float* T, int32_t n, int32_t epochs, int32_t batch, float lr,
                       int32_t seed, float* loss, void* stream);
int32_t selector_grad(void* sel, const float* X, const float* T, int32_t n, float* loss, float* grad, void* stream);
int32_t selector_predict(void* sel, const float* X, int32_t n, int32_t lmax, float* z, int32_t* rank, void* stream);
int32_t selector_save(const void* sel, const char* path);
int32_t selector_load(void* sel, const char* path);
int32_t selector_collect(Tree* t, const double* C, int64_t ldc, int32_t nocc, int32_t j0, int32_t j1,
                         int32_t max_samples, int32_t seed, float* feat, float* target, int32_t* nout, void* stream);
int32_t rank_stats(Tree* t, int64_t* hist);
bool selector_live(const void* sel);

}  // namespace occk
