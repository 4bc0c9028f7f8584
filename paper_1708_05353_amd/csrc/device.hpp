// Device-side state of a tree handle and host helpers shared by the
// standalone and batched paths.
#pragma once
#include <hip/hip_runtime.h>

#include <stdexcept>
#include <string>
#include <vector>

#include "kernels.hpp"

#define HIP_OK(x)                                                                    \
  do {                                                                               \
    hipError_t e_ = (x);                                                             \
    if (e_ != hipSuccess) throw occk::HipError(std::string(#x) + ": " + hipGetErrorString(e_)); \
  } while (0)

namespace occk {

struct HipError : std::runtime_error {
  using std::runtime_error::runtime_error;
};

// --------------------------------------------------------------------------
// host orchestration
// --------------------------------------------------------------------------
template <class T>
struct DevBuf {
  T* p = nullptr;
  size_t n = 0;
  bool own = true;   // false: a view into memory owned elsewhere (never freed here)
  // owns its allocation: freed on destruction, moved but never copied
  DevBuf() = default;
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  DevBuf(DevBuf&& o) noexcept : p(o.p), n(o.n), own(o.own) {
    o.p = nullptr;
    o.n = 0;
    o.own = true;
  }
  DevBuf& operator=(DevBuf&& o) noexcept {
    if (this != &o) {
      free();
      p = o.p;
      n = o.n;
      own = o.own;
      o.p = nullptr;
      o.n = 0;
      o.own = true;
    }
    return *this;
  }
  ~DevBuf() { free(); }
  void free() {
    if (p && own) (void)hipFree(p);
    p = nullptr;
    n = 0;
    own = true;
  }
  void view(T* ptr, size_t count) {
    free();
    p = ptr;
    n = count;
    own = false;
  }
  void upload(const std::vector<T>& v) {
    free();
    n = v.size();
    if (n == 0) return;
    HIP_OK(hipMalloc(&p, n * sizeof(T)));
    HIP_OK(hipMemcpy(p, v.data(), n * sizeof(T), hipMemcpyHostToDevice));
  }
  void alloc(size_t count) {
    if (count <= n && p) return;
    free();
    if (count == 0) return;
    HIP_OK(hipMalloc(&p, count * sizeof(T)));
    n = count;
  }
};

// Places workspace buffers one after another (256-byte aligned) in a fixed
// device region instead of allocating them; tables are copied in.  Throws
// ScratchFull when the region is too small.
struct ScratchFull : std::runtime_error {
  using std::runtime_error::runtime_error;
};

struct ScratchArena {
  char* base = nullptr;
  size_t cap = 0, off = 0;
  template <class T>
  void place(DevBuf<T>& b, size_t count) {
    const size_t bytes = (count * sizeof(T) + 255) & ~size_t(255);
    if (off + bytes > cap)
      throw ScratchFull("the workspace needs more than the " + std::to_string(cap >> 20) +
                        " MiB scratch region of the allocation-free entry point");
    b.view(reinterpret_cast<T*>(base + off), count);
    off += bytes;
  }
  template <class T>
  void upload(DevBuf<T>& b, const std::vector<T>& v) {
    place(b, v.size());
    if (!v.empty()) HIP_OK(hipMemcpy(b.p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
  }
};

struct Pass {           // one translation launch
  int ntgt = 0;
  int nent = 0;                    // CSR entries (sources over all targets)
  DevBuf<int32_t> tgt_box, src_ptr, src_box, src_op;
  std::vector<int32_t> host_op;    // host copy of src_op
  std::vector<int32_t> host_tgt;   // target (row) of each entry
  DevBuf<int32_t> ent_tgt;         // device copy of host_tgt
  DevBuf<int8_t> rank;             // per-entry rank of the learned mode
  DevBuf<float> strength;          // per-target sum of source strengths (learned mode)
};

struct DeviceState {
  int device = -1;
  // per tree
  DevBuf<double> O;               // leaf AO multipole blocks (FP64)
  DevBuf<float> Of;               // FP32 copy for the mixed paths (made on first use)
  std::vector<int64_t> O_off;     // per leaf, elements
  DevBuf<int32_t> funcs;          // concatenated leaf function lists
  std::vector<int64_t> f_off;     // per leaf
  DevBuf<OpParam> opparam;
  DevBuf<double> ops;             // FP64 operators (always generated in FP64)
  DevBuf<float> opsf;             // rounded copy for the mixed paths
  int op_sym = 0;                 // structural zeros of the operators (real_class): 0 none, 1 x axis, 2 xy plane
  // MFMA translations (Q > 9) of trees with structural zeros: components
  // grouped by class, the operators generated in that order
  DevBuf<int32_t> perm;           // [Q] component at each position (empty: none)
  DevBuf<int8_t> pcls;            // [Q] class of each position, non-decreasing
  DevBuf<double> ops_perm;        // operators in the permuted order
  DevBuf<float> opsf_perm;        // rounded copy for the mixed paths
  std::vector<Pass> up, down;     // up[k]: level depth-1-k ; down[k]: level lmin+k
  DevBuf<int32_t> occ_ptr, occ_row;
  int nbox = 0;                    // boxes on levels lmin..depth
  std::vector<int32_t> leaf_box;   // leaf -> box slot
  // per workspace shape (j batch, n_i, precision, symmetric schedule)
  int ws_jb = -1, ws_ni = -1, ws_prec = -1, ws_sym = -1;   // ws_sym: kWsPlain, kWsSym, kWsSymHT
  uint64_t ws_gen = 0;            // incremented whenever the workspace buffers are rebuilt
  // two-stream schedule (symmetric, both walks): Omega and the L2P on st2,
  // the translations on the caller's stream; the leaf Mloc and the leaf
  // Omega of odd batches go to 2 nleaf extra box rows after the Mloc
  bool ws_pipe = false;           // the box data have those extra rows
  hipStream_t st2 = nullptr;
  hipEvent_t ev_mloc[2] = {nullptr, nullptr}, ev_l2p[2] = {nullptr, nullptr}, ev_omega[2] = {nullptr, nullptr};
  hipEvent_t ev_start = nullptr, ev_join = nullptr;
  DevBuf<char> H, data;           // element type of the precision (double / float)
  DevBuf<char> HT;                // symmetric schedule: H for every column, [leaf][q][i][t]
  DevBuf<double> KB;              // per-leaf K partials, always FP64
  DevBuf<float> Cf;               // FP32 copy of C for the mixed paths
  DevBuf<GemmDesc> d_half, d_omega, d_l2p, d_ht, d_l2pt;
  DevBuf<GemmTile> t_half, t_omega, t_l2p, t_ht, t_l2pt;
  int n_half = 0, n_omega = 0, n_l2p = 0, n_ht = 0, n_l2pt = 0;
  // upward pass as one walk per subtree below each box of level upw_lroot
  // (Q <= 9; the levels above run level by level): programs
  // [upw_ptr[r], upw_ptr[r + 1])
  DevBuf<int32_t> upw_ptr;
  DevBuf<WalkStep> upw_prog;
  int upw_nroots = 0;   // 0: the level-by-level passes run instead
  int upw_nlv = 0;      // accumulator levels, D - upw_lroot
  int upw_lroot = 0;
  // downward pass as one walk per subtree below each box of level
  // dnw_lroot (Q <= 9; the levels above run level by level; not in the
  // learned-rank mode, whose ranks are per level-pass entry)
  DevBuf<int32_t> dnw_ptr;
  DevBuf<WalkStep> dnw_prog;
  int dnw_nroots = 0;   // 0: the level-by-level passes run instead
  int dnw_nlv = 0;      // accumulator levels, D - dnw_lroot + 1
  int dnw_lroot = 0;
  // mirrored L2P in 64 x 144 tiles (a whole leaf per tile), built when they
  // pad the leaves by at most a tenth more than 48-wide tiles; the
  // persistent batch kernel uses the 64 x 48 list
  DevBuf<GemmTile> t_l2ptw;
  int n_l2ptw = 0;
  // direct L2P in 144 x 64 tiles under the same rule, in chunked lists like
  // l2p_nt_start (empty when not built)
  DevBuf<GemmTile> t_l2pw;
  std::vector<int32_t> l2pw_nt_start;
  // omega and l2p: one tile list per chunk c of 4 column tiles, holding the
  // tiles with nt >= 4c, stored one after another; list c is
  // [*_nt_start[c], *_nt_start[c + 1]) and list 0 holds every tile
  std::vector<int32_t> omega_nt_start, l2p_nt_start;
  // the whole tree of a column group in LDS on chains (tree_chain_kernel;
  // Q = 9, op_sym 1): per-level stencil tables, levels lmin..depth (empty:
  // the tree is not such a chain)
  DevBuf<ChainLevel> chain;
  int chain_nlev = 0;
  int chain_nbelow = 0;   // boxes on the level above the leaves
  DevBuf<double> ops_cls;   // operators per reflection class, compact (opclass_kernel)
  int64_t ops_cls_off[4] = {0, 0, 0, 0};   // first element of each class
  size_t bytes = 0;
  // profiling: (class, start, end) event pairs recorded on the call's stream
  std::vector<hipEvent_t> ev_pool;
  size_t ev_used = 0;
  std::vector<int> ev_class;
  std::vector<size_t> ev_idx;       // first event of each recorded pair (scopes may nest)
  std::vector<int64_t> launches;
  // occupied-pair screening
  DevBuf<int32_t> home_off, home_fn;   // CSR: the functions centred in each leaf (home leaf)
  DevBuf<int32_t> hw_ptr, hw_idx;      // CSR: leaves joined to each leaf by a screened pair
  DevBuf<double> hw_val;               // largest Gaussian product factor over those pairs
  DevBuf<double> band_nrm;        // [nleaf][ni] l1 norms of C over the home functions
  DevBuf<double> band_spread;     // [nleaf][ni] the same spread over joined leaves
  DevBuf<int32_t> band_last;      // [ni] last kept i of every j
  std::vector<int32_t> band_end;  // i end of every j batch in the last screened call
  int32_t band_jb = 0;            // its j batch width
  int64_t last_band_cols = 0;     // carried columns of the last screened call
  // learned ranks
  DevBuf<float> box_norm;         // [nbox][L+1] multipole norms of the current batch
  DevBuf<int64_t> rank_hist;      // M2L entries per chosen rank (accumulated)
};

struct ProfScope {   // records a start/end event pair around a group of launches
  DeviceState* ds;
  int cls;
  hipStream_t st;
  size_t idx;
  int nlaunch;
  ProfScope(DeviceState* d, bool on, int c, hipStream_t s, int n = 1) : ds(on ? d : nullptr), cls(c), st(s), nlaunch(n) {
    if (!ds) return;
    while (ds->ev_pool.size() < ds->ev_used + 2) {
      hipEvent_t e;
      HIP_OK(hipEventCreate(&e));
      ds->ev_pool.push_back(e);
    }
    idx = ds->ev_used;
    ds->ev_used += 2;
    HIP_OK(hipEventRecord(ds->ev_pool[idx], st));
  }
  // records the end event now instead of at the end of the scope
  void close() {
    if (!ds) return;
    end();
    ds = nullptr;
  }
  ~ProfScope() {
    if (!ds) return;
    end();
  }
  void end() {
    (void)hipEventRecord(ds->ev_pool[idx + 1], st);
    ds->ev_class.push_back(cls);
    ds->ev_idx.push_back(idx);
    if (ds->launches.size() < OCCK_K_NCLASS) ds->launches.assign(OCCK_K_NCLASS, 0);
    ds->launches[cls] += nlaunch;
  }
};

size_t device_cap();
void upload_tree(Tree* t);
// arena != nullptr: place every buffer and table in that region (no allocation)
// Workspace layouts: plain (all columns), symmetric with a per-batch half
// transform beside HT (the persistent batch kernel), symmetric with the
// batch's half transform read out of HT (occk_far_K).
enum { kWsPlain = 0, kWsSym = 1, kWsSymHT = 2 };
void setup_workspace(Tree* t, int jb, int ni, int prec, int sym_mode = kWsPlain, ScratchArena* arena = nullptr);
// largest j batch width (<= 256) whose workspace fits min(cap/2, 32 GiB)
int auto_jblock(const Tree* t, int nj, int ni, size_t es, bool sym, int jmax = 256);
bool walk_tree(const Tree* t);   // both tree walks apply (chain-like trees, Q <= 9)
void ensure_mixed_operands(Tree* t, hipStream_t st);
void launch_to_float(const double* in, int64_t ldi, float* out, int64_t ldo, int64_t rows, int64_t cols,
                     hipStream_t st);
template <class T>
void launch_translate(const Tree* t, const Pass& ps, T* data, int64_t box_stride, const ColMap& cm, const T* ops,
                      hipStream_t st, const int8_t* src_rank = nullptr, const T* ops_perm = nullptr);
template <class T>
void learned_ranks(Tree* t, DeviceState* ds, const void* sel, const T* data, int64_t box_stride, const ColMap& cm,
                   hipStream_t st);
void run_upward_fp64(Tree* t, DeviceState* ds, const double* C, int64_t ldc, int i0, int i1, int j0, int j1,
                     hipStream_t st);

}  // namespace occk
