// Many systems of uneven size in one persistent launch.
//
// Each system runs the same steps as occk_far_K over all of its i and j with
// the symmetric schedule: prep (operator generation, operand conversion), the
// half transform of every column (HT), then per j batch the half transform,
// Omega over the carried columns, the upward passes, the interaction-list +
// downward passes and the two L2P contractions, and finally the K reduction.
// The host lays every task of every system into one list, grouped by stage:
// stage s holds stage s of every system that has one.  The kernel is launched
// cooperatively (all blocks co-resident); each block walks the stages in
// order and all blocks meet at one grid barrier between stages.  Within a
// stage, the blocks of XCD x (hardware block b runs on XCD b % 8) claim the
// tasks of the contiguous eighth x one at a time through an atomic counter,
// so tasks that share operand panels share an L2 and uneven tasks balance
// dynamically; a block whose eighth is drained helps with the others.  Tasks
// inside a stage are independent, the barrier orders the stages and makes
// their global-memory results visible across the XCDs, and every block
// leaves every stage after finitely many claims, so every wave exits.
#include <hip/hip_cooperative_groups.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstring>
#include <stdexcept>
#include <vector>

#include "device.hpp"

namespace occk {

enum BTaskType : int16_t { kTOpgen = 0, kTConvert, kTHT, kTHalf, kTOmega, kTTrans, kTL2P, kTL2PT, kTReduce };

struct BTask {
  int16_t type, sys;
  int32_t a, b;          // type-specific (tile / op / pass / row-chunk ranges)
  int32_t kb, pad;       // j batch
};

struct BPass {
  const int32_t* tgt_box;
  const int32_t* src_ptr;
  const int32_t* src_box;
  const int32_t* src_op;
  int32_t ntgt, pad;
};

struct BSys {
  const GemmDesc* d_half;
  const GemmTile* t_half;
  const GemmDesc* d_omega;
  const GemmTile* t_omega;
  const GemmDesc* d_l2p;
  const GemmTile* t_l2p;
  const GemmDesc* d_ht;
  const GemmTile* t_ht;
  const GemmDesc* d_l2pt;
  const GemmTile* t_l2pt;
  const double* Cin;     // caller's C for this run
  int64_t ldcin;
  void* Cf;              // FP32 copy (mixed modes)
  double* K;             // caller's K
  int64_t ldk;
  void* data;
  int64_t box_stride, ncol;
  const OpParam* opparam;
  double* ops;
  float* opsf;
  double* KB;
  const int32_t* occ_ptr;
  const int32_t* occ_row;
  int32_t nbasis, nocc, L, Q, KS, pass0, jb, pad;
};

struct BatchPlan {
  uint32_t magic = 0x62617463u;
  int nsys = 0, prec = 0, L = 0, Q = 0;
  int jblock = 0;                // requested j batch width (0: per-system automatic)
  std::vector<Tree*> trees;
  std::vector<int> nocc, jb;
  std::vector<uint64_t> ws_gen;  // workspace generation of every tree when the tables were built
  // device tables
  DevBuf<BSys> sys;
  DevBuf<BPass> passes;
  DevBuf<BTask> tasks;
  DevBuf<int32_t> stage_ptr;   // tasks of stage s: [stage_ptr[s], stage_ptr[s+1])
  DevBuf<uint64_t> stage_clk;  // wall clock after each stage of the last launch (entry 0: start)
  DevBuf<int> claim;           // per (stage, eighth) task claim counters, zeroed before each launch
  std::vector<int16_t> stage_type;  // task type of the largest system's task in each stage
  int ntasks = 0, nstage = 0;
  int max_blocks_per_cu = 1;   // co-residency limit of the kernel
  std::vector<BSys> host_sys;
  std::vector<BPass> host_passes;
  // tunables
  int blocks_per_cu = 2, gemm_group = 1, trans_group = 1;
  int tuned = 0;
  int ncu = 0;
  std::vector<double> tune_ms;
};

static constexpr int64_t kConvertRows = 64;
static constexpr int kReduceRows = 8;
static constexpr int kVecCols = 2;   // columns per thread of the small-Q translation tiles

// carried columns per translation block
__host__ __device__ static inline int trans_block_cols(int Q) { return Q <= 9 ? 256 * kVecCols : 256; }

// --------------------------------------------------------------------------
// device side
// --------------------------------------------------------------------------
// Shared memory of the persistent kernel: one task at a time uses it.
template <int MODE>
union BatchSmem {
  GemmSmem<MODE, GemmSquare> sq;
  GemmSmem<MODE, GemmRows48> rows;
  GemmSmem<MODE, GemmCols48> cols;
};

// QV > 0: translations as exact-size vector FMAs for Q = QV (L <= 2);
// QV == 0: MFMA translation tiles with MT row tiles.
template <int MODE, int MT, int QV>
__device__ __forceinline__ void batch_body(const BTask* __restrict__ tasks, const int32_t* __restrict__ stage_ptr,
                                           int nstage, const BSys* __restrict__ sys,
                                           const BPass* __restrict__ passes, int gemm_group, int trans_group,
                                           uint64_t* __restrict__ stage_clk, int* __restrict__ claim,
                                           BatchSmem<MODE>& sm) {
  using T = typename ModeT<MODE>::T;
  cooperative_groups::grid_group grid = cooperative_groups::this_grid();
  const bool clock_block = stage_clk && blockIdx.x == 0 && threadIdx.x == 0;
  if (clock_block) stage_clk[0] = wall_clock64();
  const int tid = threadIdx.x;
  const int xcd = int(blockIdx.x % 8);
  __shared__ int s_task;
  for (int stage = 0; stage < nstage; ++stage) {
    const int s0 = as_const(stage_ptr)[stage], ns = as_const(stage_ptr)[stage + 1] - s0;
    // Eighth y of the stage's tasks is claimed through counter (stage, y); a
    // block drains its own XCD's eighth first, then the others in turn.
    // Every claim is an atomic increment, so each task runs exactly once,
    // and each counter passes its eighth's size after finitely many claims,
    // so every block reaches the barrier.
    for (int v = 0; v < 8; ++v) {
    const int y = (xcd + v) & 7;
    const int lo = s0 + int(int64_t(ns) * y / 8), hi = s0 + int(int64_t(ns) * (y + 1) / 8);
    for (;;) {
      if (tid == 0) s_task = lo + atomicAdd(&claim[stage * 8 + y], 1);
      __syncthreads();
      const int k = s_task;
      __syncthreads();   // every thread has read s_task before it is overwritten
      if (k >= hi) break;
      const BTask tk = load_const(tasks + k);
      const BSys S = load_const(sys + tk.sys);
      const T* Cg = MODE == kModeF64 ? reinterpret_cast<const T*>(S.Cin) : reinterpret_cast<const T*>(S.Cf);
      const int64_t ldcg = MODE == kModeF64 ? S.ldcin : int64_t(S.nocc);
      const int n = S.nocc, jb = S.jb;
      const int jrel = tk.kb * jb;             // first j of the batch = first carried i
      GemmRun run{};
      switch (tk.type) {
        case kTConvert: {   // rows [a, b) of C -> FP32
          gbl<float>* out = as_global(static_cast<float*>(S.Cf));
          const gbl<const double>* cin = as_global(S.Cin);
          const int64_t nel = int64_t(tk.b - tk.a) * n;
          for (int64_t e = tid; e < nel; e += 256) {
            const int64_t r = tk.a + e / n, c = e % n;
            out[r * n + c] = float(cin[r * S.ldcin + c]);
          }
          break;
        }
        case kTHT:
          run.blim = n;
          for (int g = tk.a; g < tk.b; ++g) {
            const GemmTile tl = load_const(S.t_ht + g);
            gemm_tile<MODE, true, true, T, GemmRows48>(load_const(S.d_ht + tl.prob), tl.mt, tl.nt, Cg, ldcg, run, sm.rows);
          }
          break;
        case kTHalf:
          run.boff = jrel;
          run.blim = n;
          for (int g = tk.a; g < tk.b; ++g) {
            const GemmTile tl = load_const(S.t_half + g);
            gemm_tile<MODE, true, true, T, GemmRows48>(load_const(S.d_half + tl.prob), tl.mt, tl.nt, Cg, ldcg, run, sm.rows);
          }
          break;
        case kTOmega:
          run.blim = n;
          for (int g = tk.a; g < tk.b; ++g) {
            const GemmTile tl = load_const(S.t_omega + g);
            gemm_tile<MODE, false, true, T>(load_const(S.d_omega + tl.prob), tl.mt, tl.nt, Cg, ldcg, run, sm.sq);
          }
          break;
        case kTTrans: {     // pass a, logical blocks [b, b + trans_group)
          const BPass P = load_const(passes + S.pass0 + tk.a);
          const ColMap cm{S.ncol, int64_t(n), int64_t(jrel), int64_t(jb) * (n - jrel), 0};
          const int64_t nct = (cm.nvalid + trans_block_cols(S.Q) - 1) / trans_block_cols(S.Q);
          const int64_t nblocks = nct * P.ntgt;
          const int64_t e1 = (nblocks < int64_t(tk.b) + trans_group) ? nblocks : int64_t(tk.b) + trans_group;
          const T* ops = MODE == kModeF64 ? reinterpret_cast<const T*>(S.ops) : reinterpret_cast<const T*>(S.opsf);
          for (int64_t lb = tk.b; lb < e1; ++lb) {
            if constexpr (QV > 0)
              translate_vec_tile<T, QV, kVecCols, 0, false>(static_cast<T*>(S.data), S.box_stride, cm, S.KS, P.tgt_box,
                                                  P.src_ptr, P.src_box, P.src_op, S.ops, int(lb % P.ntgt), lb / P.ntgt);
            else
              translate_tile<T, MT, (sizeof(BatchSmem<MODE>) >= sizeof(T) * MT * 4 * MT * 64)>(
                  static_cast<T*>(S.data), S.box_stride, cm, S.Q, S.KS, P.tgt_box, P.src_ptr, P.src_box, P.src_op,
                  ops, int(lb % P.ntgt), lb / P.ntgt, nullptr, reinterpret_cast<T*>(&sm));
          }
          break;
        }
        case kTL2P:
          run.accumulate = tk.kb > 0 ? 1 : 0;
          run.nlo = jrel;
          for (int g = tk.a; g < tk.b; ++g) {
            const GemmTile tl = load_const(S.t_l2p + g);
            gemm_tile<MODE, true, false, double, GemmRows48>(load_const(S.d_l2p + tl.prob), tl.mt, tl.nt, Cg, ldcg, run, sm.rows);
          }
          break;
        case kTL2PT:
          run.accumulate = 1;
          run.koff = jrel + jb;
          run.coff = jrel;
          run.mlim = (n - jrel < jb) ? n - jrel : jb;
          for (int g = tk.a; g < tk.b; ++g) {
            const GemmTile tl = load_const(S.t_l2pt + g);
            gemm_tile<MODE, true, false, double, GemmCols48>(load_const(S.d_l2pt + tl.prob), tl.mt, tl.nt, Cg, ldcg, run, sm.cols);
          }
          break;
        case kTReduce: {    // rows [a, b)
          const int64_t nel = int64_t(tk.b - tk.a) * n;
          for (int64_t e = tid; e < nel; e += 256)
            reduce_elem(S.KB, n, S.occ_ptr, S.occ_row, S.K, S.ldk, 0, 0, int(tk.a + e / n), e % n);
          break;
        }
        default:
          break;
      }
      __syncthreads();   // shared memory is reused by the block's next task
    }
    }
    grid.sync();
    if (clock_block) stage_clk[stage + 1] = wall_clock64();
  }
}

// One translation row tile (L <= 3): FP64 / FP32 at most 128 VGPRs (4 waves
// per SIMD), the split-BF16 modes at most 168 (3 waves per SIMD; their GEMM
// tiles hold bf16 fragments of three planes), which the union of all task
// paths fits without spills.  More row tiles (L >= 4) keep the compiler's
// own allocation, which is free of spills up to L = 8.
template <int MODE, int MT, int QV>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4, 8))) void batch_kernel_w4(
    const BTask* __restrict__ tasks, const int32_t* __restrict__ stage_ptr, int nstage, const BSys* __restrict__ sys,
    const BPass* __restrict__ passes, int gemm_group, int trans_group, uint64_t* __restrict__ stage_clk,
    int* __restrict__ claim) {
  __shared__ BatchSmem<MODE> sm;
  batch_body<MODE, MT, QV>(tasks, stage_ptr, nstage, sys, passes, gemm_group, trans_group, stage_clk, claim, sm);
}

template <int MODE, int MT, int QV>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3, 8))) void batch_kernel_w3(
    const BTask* __restrict__ tasks, const int32_t* __restrict__ stage_ptr, int nstage, const BSys* __restrict__ sys,
    const BPass* __restrict__ passes, int gemm_group, int trans_group, uint64_t* __restrict__ stage_clk,
    int* __restrict__ claim) {
  __shared__ BatchSmem<MODE> sm;
  batch_body<MODE, MT, QV>(tasks, stage_ptr, nstage, sys, passes, gemm_group, trans_group, stage_clk, claim, sm);
}

template <int MODE, int MT, int QV>
__global__ __launch_bounds__(256) void batch_kernel(const BTask* __restrict__ tasks,
                                                    const int32_t* __restrict__ stage_ptr, int nstage,
                                                    const BSys* __restrict__ sys, const BPass* __restrict__ passes,
                                                    int gemm_group, int trans_group,
                                                    uint64_t* __restrict__ stage_clk, int* __restrict__ claim) {
  __shared__ BatchSmem<MODE> sm;
  batch_body<MODE, MT, QV>(tasks, stage_ptr, nstage, sys, passes, gemm_group, trans_group, stage_clk, claim, sm);
}

static __global__ void zero_i32_kernel(int* __restrict__ p, int n) {
  for (int i = threadIdx.x; i < n; i += blockDim.x) p[i] = 0;
}

// --------------------------------------------------------------------------
// host side
// --------------------------------------------------------------------------
static void build_tasks(BatchPlan& bp) {
  std::vector<BTask> tasks;
  struct Stage {
    std::vector<BTask> t;
  };
  std::vector<std::vector<Stage>> st(bp.nsys);
  int maxst = 0;
  for (int k = 0; k < bp.nsys; ++k) {
    Tree* t = bp.trees[k];
    DeviceState* ds = t->dev;
    const BSys& S = bp.host_sys[k];
    const int n = S.nocc, jb = S.jb;
    auto& v = st[k];
    const int16_t sk = int16_t(k);
    Stage prep;
    if (bp.prec != OCCK_PREC_FP64)
      for (int64_t r = 0; r < S.nbasis; r += kConvertRows)
        prep.t.push_back(
            {kTConvert, sk, int32_t(r), int32_t(std::min<int64_t>(S.nbasis, r + kConvertRows)), 0, 0});
    v.push_back(prep);
    auto gemm_stage = [&](int16_t type, int g0, int g1, int kb) {
      Stage s;
      for (int g = g0; g < g1; g += bp.gemm_group)
        s.t.push_back({type, sk, g, std::min(g1, g + bp.gemm_group), kb, 0});
      v.push_back(s);
    };
    gemm_stage(kTHT, 0, ds->n_ht, 0);
    const int nblk = (n + jb - 1) / jb;
    const int np = int(ds->up.size() + ds->down.size());
    const int tbc = trans_block_cols(S.Q);
    for (int kb = 0; kb < nblk; ++kb) {
      const int jrel = kb * jb;
      const int ch = (jrel / 64) / 4;             // first chunk of 4 column tiles touching i >= jrel
      gemm_stage(kTHalf, 0, ds->n_half, kb);
      gemm_stage(kTOmega, ds->omega_nt_start[size_t(ch)], ds->omega_nt_start[size_t(ch) + 1], kb);
      const int64_t nct = (int64_t(jb) * (n - jrel) + tbc - 1) / tbc;
      for (int p = 0; p < np; ++p) {
        const BPass& P = bp.host_passes[size_t(S.pass0 + p)];
        if (nct * P.ntgt > int64_t(0x7fffffff)) throw std::invalid_argument("batch: translation grid too large");
        Stage s;
        for (int64_t lb = 0; lb < nct * P.ntgt; lb += bp.trans_group)
          s.t.push_back({kTTrans, sk, p, int32_t(lb), kb, 0});
        v.push_back(s);
      }
      gemm_stage(kTL2P, ds->l2p_nt_start[size_t(ch)], ds->l2p_nt_start[size_t(ch) + 1], kb);
      if (jrel + jb < n) gemm_stage(kTL2PT, 0, ds->n_l2pt, kb);
    }
    Stage red;
    for (int r = 0; r < S.nbasis; r += kReduceRows)
      red.t.push_back({kTReduce, sk, r, std::min(S.nbasis, r + kReduceRows), 0, 0});
    v.push_back(red);
    maxst = std::max(maxst, int(v.size()));
  }
  // stage-grouped list: stage s of every system that has one
  bp.stage_type.assign(size_t(maxst), -1);
  for (int k = 0; k < bp.nsys; ++k)
    for (int s = 0; s < int(st[k].size()); ++s)
      if (bp.stage_type[size_t(s)] < 0 && !st[k][s].t.empty()) bp.stage_type[size_t(s)] = st[k][s].t[0].type;
  std::vector<int32_t> sptr{0};
  for (int s = 0; s < maxst; ++s) {
    for (int k = 0; k < bp.nsys; ++k)
      if (s < int(st[k].size())) tasks.insert(tasks.end(), st[k][s].t.begin(), st[k][s].t.end());
    if (tasks.size() > size_t(0x7fffffff)) throw std::invalid_argument("batch: too many tasks");
    sptr.push_back(int32_t(tasks.size()));
  }
  bp.ntasks = int(tasks.size());
  bp.nstage = maxst;
  bp.tasks.upload(tasks);
  bp.stage_ptr.upload(sptr);
}

static void prepare(BatchPlan& bp, hipStream_t st) {
  const bool mixed = bp.prec != OCCK_PREC_FP64;
  const size_t es = mixed ? 4 : 8;
  bp.host_sys.assign(bp.nsys, BSys{});
  bp.ws_gen.assign(size_t(bp.nsys), 0);
  bp.jb.assign(size_t(bp.nsys), 0);
  bp.host_passes.clear();
  for (int k = 0; k < bp.nsys; ++k) {
    Tree* t = bp.trees[k];
    if (!t->dev) upload_tree(t);
    DeviceState* ds = t->dev;
    if (mixed) ensure_mixed_operands(t, st);
    // translation operators depend on the geometry only: generated once per
    // plan (FP64 by recurrence, then the rounded FP32 copy), not per run
    hipLaunchKernelGGL(opgen_kernel, dim3(unsigned(t->ops.size())), dim3(64), 0, st, ds->opparam.p, ds->ops.p, t->L,
                       t->Q);
    HIP_OK(hipGetLastError());
    if (mixed) launch_to_float(ds->ops.p, 0, ds->opsf.p, 0, 1, int64_t(ds->ops.n), st);
    const int n = bp.nocc[k];
    const int jb = bp.jblock > 0 ? std::min(bp.jblock, n) : auto_jblock(t, n, n, es, true);
    setup_workspace(t, jb, n, bp.prec, kWsSym);
    if (mixed) ds->Cf.alloc(size_t(t->nbasis) * n);
    bp.ws_gen[size_t(k)] = ds->ws_gen;
    bp.jb[size_t(k)] = jb;
    BSys& S = bp.host_sys[k];
    S.d_half = ds->d_half.p;
    S.t_half = ds->t_half.p;
    S.d_omega = ds->d_omega.p;
    S.t_omega = ds->t_omega.p;
    S.d_l2p = ds->d_l2p.p;
    S.t_l2p = ds->t_l2p.p;
    S.d_ht = ds->d_ht.p;
    S.t_ht = ds->t_ht.p;
    S.d_l2pt = ds->d_l2pt.p;
    S.t_l2pt = ds->t_l2pt.p;
    S.Cf = mixed ? ds->Cf.p : nullptr;
    S.data = ds->data.p;
    S.ncol = int64_t(jb) * n;
    S.box_stride = int64_t(t->Q) * S.ncol;
    S.opparam = ds->opparam.p;
    S.ops = ds->ops.p;
    S.opsf = mixed ? ds->opsf.p : nullptr;
    S.KB = ds->KB.p;
    S.occ_ptr = ds->occ_ptr.p;
    S.occ_row = ds->occ_row.p;
    S.nbasis = t->nbasis;
    S.nocc = n;
    S.L = t->L;
    S.Q = t->Q;
    S.KS = ksteps_of(t->Q);
    S.jb = jb;
    S.pass0 = int(bp.host_passes.size());
    for (const Pass& p : ds->up)
      bp.host_passes.push_back({p.tgt_box.p, p.src_ptr.p, p.src_box.p, p.src_op.p, p.ntgt, 0});
    for (const Pass& p : ds->down)
      bp.host_passes.push_back({p.tgt_box.p, p.src_ptr.p, p.src_box.p, p.src_op.p, p.ntgt, 0});
  }
  bp.passes.upload(bp.host_passes);
  bp.sys.upload(bp.host_sys);
  build_tasks(bp);
}

template <int MODE, int MT, int QV>
static const void* kernel_of() {
  if constexpr ((MODE == kModeF64 || MODE == kModeF32) && MT == 1)
    return reinterpret_cast<const void*>(batch_kernel_w4<MODE, MT, QV>);
  else if constexpr (MT == 1)
    return reinterpret_cast<const void*>(batch_kernel_w3<MODE, MT, QV>);
  else
    return reinterpret_cast<const void*>(batch_kernel<MODE, MT, QV>);
}

template <int MODE>
static const void* kernel_for_q(int Q) {
  switch (Q) {
    case 1: return kernel_of<MODE, 1, 1>();
    case 4: return kernel_of<MODE, 1, 4>();
    case 9: return kernel_of<MODE, 1, 9>();
    default: break;
  }
  switch (mtiles_of(Q)) {
    case 1: return kernel_of<MODE, 1, 0>();
    case 2: return kernel_of<MODE, 2, 0>();
    case 3: return kernel_of<MODE, 3, 0>();
    case 4: return kernel_of<MODE, 4, 0>();
    case 5: return kernel_of<MODE, 5, 0>();
    case 6: return kernel_of<MODE, 6, 0>();
    default: throw std::invalid_argument("unsupported Q");
  }
}

static const void* batch_kernel_for(const BatchPlan& bp) {
  switch (bp.prec) {
    case OCCK_PREC_FP64: return kernel_for_q<kModeF64>(bp.Q);
    case OCCK_PREC_FP32: return kernel_for_q<kModeF32>(bp.Q);
    case OCCK_PREC_BF16X3: return kernel_for_q<kModeBF16x3>(bp.Q);
    default: return kernel_for_q<kModeBF16x6>(bp.Q);
  }
}

// The grid barrier relies on every block being resident.  Residency is
// established from the occupancy query, which accounts for registers and
// LDS; a kernel that spills to scratch memory is refused so that no other
// resource can hold blocks back.
static void check_kernel(BatchPlan& bp) {
  const void* kern = batch_kernel_for(bp);
  hipFuncAttributes fa;
  HIP_OK(hipFuncGetAttributes(&fa, kern));
  if (fa.localSizeBytes > 0)
    throw std::invalid_argument("batch: the persistent kernel for this lmax and precision spills registers; "
                                "batched launches need a spill-free kernel");
  int per_cu = 0;
  HIP_OK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, 256, 0));
  if (per_cu < 1) throw HipError("batch kernel cannot be resident");
  bp.max_blocks_per_cu = per_cu;
}

static void launch(BatchPlan& bp, hipStream_t st) {
  const void* kern = batch_kernel_for(bp);
  // a multiple of 8 blocks (one share per XCD), never above the co-resident count
  const int grid = ((bp.ncu * std::min(bp.blocks_per_cu, bp.max_blocks_per_cu)) / 8) * 8;
  if (grid < 8) throw HipError("batch kernel: fewer than 8 co-resident blocks");
  const BTask* tasks = bp.tasks.p;
  const int32_t* sptr = bp.stage_ptr.p;
  int nstage = bp.nstage;
  const BSys* sys = bp.sys.p;
  const BPass* passes = bp.passes.p;
  int gg = bp.gemm_group, tg = bp.trans_group;
  bp.stage_clk.alloc(size_t(bp.nstage) + 1);
  uint64_t* clk = bp.stage_clk.p;
  bp.claim.alloc(size_t(bp.nstage) * 8);
  int* claim = bp.claim.p;
  hipLaunchKernelGGL(zero_i32_kernel, dim3(1), dim3(256), 0, st, claim, bp.nstage * 8);   // kernel, not a memset node
  HIP_OK(hipGetLastError());
  void* args[] = {&tasks, &sptr, &nstage, &sys, &passes, &gg, &tg, &clk, &claim};
  HIP_OK(hipLaunchCooperativeKernel(kern, dim3(unsigned(grid)), dim3(256), args, 0, st));
}

static void set_io(BatchPlan& bp, const double* const* C, const int64_t* ldc, double* const* K, const int64_t* ldk) {
  bool changed = false;
  for (int k = 0; k < bp.nsys; ++k) {
    BSys& S = bp.host_sys[k];
    if (S.Cin != C[k] || S.ldcin != ldc[k] || S.K != K[k] || S.ldk != ldk[k]) changed = true;
    S.Cin = C[k];
    S.ldcin = ldc[k];
    S.K = K[k];
    S.ldk = ldk[k];
  }
  if (changed)   // synchronous: the table must not change under a queued copy
    HIP_OK(hipMemcpy(bp.sys.p, bp.host_sys.data(), bp.host_sys.size() * sizeof(BSys), hipMemcpyHostToDevice));
}

// --------------------------------------------------------------------------
// entry points (called from abi.cpp after validation)
// --------------------------------------------------------------------------
int32_t batch_create(int nsys, Tree* const* trees, const int32_t* nocc, int prec, int jblock, void** out) {
  BatchPlan* bp = new BatchPlan();
  try {
    bp->nsys = nsys;
    bp->prec = prec;
    bp->jblock = jblock;
    bp->trees.assign(trees, trees + nsys);
    bp->nocc.assign(nocc, nocc + nsys);
    bp->L = trees[0]->L;
    bp->Q = trees[0]->Q;
    int dev = 0;
    HIP_OK(hipGetDevice(&dev));
    hipDeviceProp_t prop;
    HIP_OK(hipGetDeviceProperties(&prop, dev));
    bp->ncu = prop.multiProcessorCount;
    check_kernel(*bp);
    bp->blocks_per_cu = bp->max_blocks_per_cu;   // untuned default: every co-resident block
    prepare(*bp, nullptr);
    HIP_OK(hipDeviceSynchronize());
  } catch (const HipError& e) {
    delete bp;
    set_error(e.what());
    return OCCK_EHIP;
  } catch (const std::bad_alloc&) {
    delete bp;
    set_error("batch: device allocation failed or exceeds OCCK_MAX_DEVICE_BYTES");
    return OCCK_ENOMEM;
  } catch (const std::invalid_argument& e) {
    delete bp;
    set_error(e.what());
    return OCCK_EINVAL;
  }
  *out = bp;
  return OCCK_OK;
}

// A standalone occk_far_K on one of the trees may have replaced its
// workspace; the plan then rebuilds its tables (synchronously).
static void revalidate(BatchPlan& bp) {
  bool stale = false;
  for (int k = 0; k < bp.nsys; ++k) {
    const DeviceState* ds = bp.trees[k]->dev;
    if (!ds || ds->ws_jb != bp.jb[size_t(k)] || ds->ws_ni != bp.nocc[k] || ds->ws_prec != bp.prec ||
        ds->ws_sym != kWsSym || ds->ws_gen != bp.ws_gen[size_t(k)] ||
        (bp.prec != OCCK_PREC_FP64 && ds->Cf.p != bp.host_sys[k].Cf))
      stale = true;
  }
  if (!stale) return;
  HIP_OK(hipDeviceSynchronize());
  prepare(bp, nullptr);
  HIP_OK(hipDeviceSynchronize());
}

int32_t batch_run(void* plan, const double* const* C, const int64_t* ldc, double* const* K, const int64_t* ldk,
                  void* stream) {
  BatchPlan& bp = *static_cast<BatchPlan*>(plan);
  try {
    revalidate(bp);
    set_io(bp, C, ldc, K, ldk);
    launch(bp, reinterpret_cast<hipStream_t>(stream));
  } catch (const HipError& e) {
    set_error(e.what());
    return OCCK_EHIP;
  } catch (const std::bad_alloc&) {
    set_error("batch: device allocation failed or exceeds OCCK_MAX_DEVICE_BYTES");
    return OCCK_ENOMEM;
  } catch (const std::invalid_argument& e) {
    set_error(e.what());
    return OCCK_EINVAL;
  }
  return OCCK_OK;
}

// Times every candidate (blocks per CU, GEMM tiles per task, translation
// column tiles per task) once after a warm-up and keeps the fastest.
int32_t batch_tune(void* plan, const double* const* C, const int64_t* ldc, double* const* K, const int64_t* ldk,
                   void* stream, int32_t* choice) {
  BatchPlan& bp = *static_cast<BatchPlan*>(plan);
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  std::vector<int> bpc{2, 4, bp.max_blocks_per_cu};   // blocks per CU (capped at the co-resident count)
  std::sort(bpc.begin(), bpc.end());
  bpc.erase(std::unique(bpc.begin(), bpc.end()), bpc.end());
  const int gg[] = {1, 2};
  const int tg[] = {1, 4};
  double best = 1e300;
  int bb = bp.blocks_per_cu, bg = 1, bt = 1;
  bp.tune_ms.clear();
  try {
    revalidate(bp);
    set_io(bp, C, ldc, K, ldk);
    hipEvent_t e0, e1;
    HIP_OK(hipEventCreate(&e0));
    HIP_OK(hipEventCreate(&e1));
    for (int b : bpc)
      for (int g : gg)
        for (int tt : tg) {
          bp.blocks_per_cu = b;
          if (g != bp.gemm_group || tt != bp.trans_group || bp.ntasks == 0) {
            bp.gemm_group = g;
            bp.trans_group = tt;
            build_tasks(bp);
          }
          launch(bp, st);   // warm-up
          HIP_OK(hipEventRecord(e0, st));
          launch(bp, st);
          HIP_OK(hipEventRecord(e1, st));
          HIP_OK(hipEventSynchronize(e1));
          float ms = 0.f;
          HIP_OK(hipEventElapsedTime(&ms, e0, e1));
          bp.tune_ms.push_back(ms);
          if (ms < best) {
            best = ms;
            bb = b;
            bg = g;
            bt = tt;
          }
        }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    bp.blocks_per_cu = bb;
    bp.gemm_group = bg;
    bp.trans_group = bt;
    build_tasks(bp);
    bp.tuned = 1;
  } catch (const HipError& e) {
    set_error(e.what());
    return OCCK_EHIP;
  } catch (const std::invalid_argument& e) {
    set_error(e.what());
    return OCCK_EINVAL;
  }
  if (choice) {
    choice[0] = bb;
    choice[1] = bg;
    choice[2] = bt;
  }
  return OCCK_OK;
}

int32_t batch_free(void* plan) {
  BatchPlan* bp = static_cast<BatchPlan*>(plan);
  (void)hipDeviceSynchronize();
  bp->sys.free();
  bp->passes.free();
  bp->tasks.free();
  bp->stage_ptr.free();
  bp->stage_clk.free();
  bp->claim.free();
  bp->magic = 0;
  delete bp;
  return OCCK_OK;
}

// Per-stage durations (ms) of the last launch and the task type of each
// stage (synchronises the device).
int32_t batch_stage_times(void* plan, double* ms, int32_t* type, int cap, int32_t* nstage) {
  BatchPlan& bp = *static_cast<BatchPlan*>(plan);
  try {
    if (nstage) *nstage = bp.nstage;
    if (!bp.stage_clk.p || cap <= 0) return OCCK_OK;
    HIP_OK(hipDeviceSynchronize());
    std::vector<uint64_t> clk(size_t(bp.nstage) + 1);
    HIP_OK(hipMemcpy(clk.data(), bp.stage_clk.p, clk.size() * sizeof(uint64_t), hipMemcpyDeviceToHost));
    int dev = 0, khz = 0;
    HIP_OK(hipGetDevice(&dev));
    HIP_OK(hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev));
    if (khz <= 0) throw HipError("wall clock rate unknown");
    for (int s = 0; s < std::min(cap, bp.nstage); ++s) {
      if (ms) ms[s] = double(clk[size_t(s) + 1] - clk[size_t(s)]) / double(khz);
      if (type) type[s] = bp.stage_type[size_t(s)];
    }
  } catch (const HipError& e) {
    set_error(e.what());
    return OCCK_EHIP;
  }
  return OCCK_OK;
}

int32_t batch_shape(const void* plan, int32_t* nsys, int32_t* nocc, int cap, int32_t* tuned) {
  const BatchPlan& bp = *static_cast<const BatchPlan*>(plan);
  if (nsys) *nsys = bp.nsys;
  if (nocc)
    for (int k = 0; k < std::min(cap, bp.nsys); ++k) nocc[k] = bp.nocc[k];
  if (tuned) {
    tuned[0] = bp.blocks_per_cu;
    tuned[1] = bp.gemm_group;
    tuned[2] = bp.trans_group;
    tuned[3] = bp.ntasks;
    tuned[4] = bp.nstage;
    tuned[5] = bp.max_blocks_per_cu;
  }
  return OCCK_OK;
}

}  // namespace occk
