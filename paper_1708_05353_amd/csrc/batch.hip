// Many systems of uneven size in one persistent launch.
//
// Each system runs the same steps as occk_far_K with a single j batch (all
// i, all j): prep (operator generation, operand conversion), half transform,
// Omega, the upward passes, the interaction-list + downward passes, L2P and
// the K reduction.  The host lays every task of every system into one list,
// grouped by stage: stage s holds stage s of every system that has one.  The
// kernel is launched cooperatively (all blocks co-resident); each block walks
// the stages in order, takes the tasks of the current stage with a static
// stride (block b: tasks b, b + grid, ...), and all blocks meet at one grid
// barrier between stages.  Tasks inside a stage are independent, the barrier
// orders the stages and makes their global-memory results visible across the
// XCDs, and every block executes the same bounded loop, so every wave exits.
#include <hip/hip_cooperative_groups.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstring>
#include <vector>

#include "device.hpp"

namespace occk {

enum BTaskType : int16_t { kTOpgen = 0, kTConvert, kTHalf, kTOmega, kTTrans, kTL2P, kTReduce };

struct BTask {
  int16_t type, sys;
  int32_t a, b;          // type-specific (tile / op / pass / row-chunk ranges)
};

struct BPass {
  const int32_t* tgt_box;
  const int32_t* src_ptr;
  const int32_t* src_box;
  const int32_t* src_op;
  int32_t ntgt, pad;
  int64_t nblocks;       // (column tiles) x (targets)
};

struct BSys {
  const GemmDesc* d_half;
  const GemmTile* t_half;
  const GemmDesc* d_omega;
  const GemmTile* t_omega;
  const GemmDesc* d_l2p;
  const GemmTile* t_l2p;
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
  int32_t nbasis, nocc, L, Q, KS, pass0;
};

struct BatchPlan {
  uint32_t magic = 0x62617463u;
  int nsys = 0, prec = 0, L = 0, Q = 0;
  std::vector<Tree*> trees;
  std::vector<int> nocc;
  std::vector<uint64_t> ws_gen;  // workspace generation of every tree when the tables were built
  // device tables
  DevBuf<BSys> sys;
  DevBuf<BPass> passes;
  DevBuf<BTask> tasks;
  DevBuf<int32_t> stage_ptr;   // tasks of stage s: [stage_ptr[s], stage_ptr[s+1])
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

// --------------------------------------------------------------------------
// device side
// --------------------------------------------------------------------------
template <int MODE, int MT>
__global__ __launch_bounds__(256) void batch_kernel(const BTask* __restrict__ tasks,
                                                    const int32_t* __restrict__ stage_ptr, int nstage,
                                                    const BSys* __restrict__ sys, const BPass* __restrict__ passes,
                                                    int gemm_group, int trans_group) {
  using T = typename ModeT<MODE>::T;
  __shared__ GemmSmem<MODE> sm;
  __shared__ Cplx tab[(2 * kMaxL + 1) * (2 * kMaxL + 2) / 2];
  cooperative_groups::grid_group grid = cooperative_groups::this_grid();
  const int tid = threadIdx.x;
  for (int stage = 0; stage < nstage; ++stage) {
    for (int k = stage_ptr[stage] + blockIdx.x; k < stage_ptr[stage + 1]; k += gridDim.x) {
      const BTask tk = tasks[k];
      const BSys& S = sys[tk.sys];
      const T* Cg = MODE == kModeF64 ? reinterpret_cast<const T*>(S.Cin) : reinterpret_cast<const T*>(S.Cf);
      const int64_t ldcg = MODE == kModeF64 ? S.ldcin : int64_t(S.nocc);
      const int64_t opsz = int64_t(mtiles_of(S.Q)) * ksteps_of(S.Q) * 64;
      GemmRun gather{};   // one j batch of all nocc columns: B gathered from C columns [0, nocc)
      gather.blim = S.nocc;
      const ColMap cm{S.ncol, int64_t(S.nocc), 0, S.ncol};
      switch (tk.type) {
        case kTOpgen:
          opgen_one(S.opparam[tk.a], S.ops + int64_t(tk.a) * opsz,
                    MODE == kModeF64 ? nullptr : S.opsf + int64_t(tk.a) * opsz, S.L, S.Q, tab, tid, 256);
          break;
        case kTConvert: {   // rows [a, b) of C -> FP32
          float* out = static_cast<float*>(S.Cf);
          const int64_t n = int64_t(tk.b - tk.a) * S.nocc;
          for (int64_t e = tid; e < n; e += 256) {
            const int64_t r = tk.a + e / S.nocc, c = e % S.nocc;
            out[r * S.nocc + c] = float(S.Cin[r * S.ldcin + c]);
          }
          break;
        }
        case kTHalf:
          for (int g = tk.a; g < tk.b; ++g) {
            const GemmTile tl = S.t_half[g];
            gemm_tile<MODE, true, T>(S.d_half[tl.prob], tl.mt, tl.nt, Cg, ldcg, gather, sm);
          }
          break;
        case kTOmega:
          for (int g = tk.a; g < tk.b; ++g) {
            const GemmTile tl = S.t_omega[g];
            gemm_tile<MODE, false, T>(S.d_omega[tl.prob], tl.mt, tl.nt, Cg, ldcg, gather, sm);
          }
          break;
        case kTTrans: {     // pass a, logical blocks [b, b + trans_group)
          const BPass& P = passes[S.pass0 + tk.a];
          const int64_t e1 = (P.nblocks < int64_t(tk.b) + trans_group) ? P.nblocks : int64_t(tk.b) + trans_group;
          const T* ops = MODE == kModeF64 ? reinterpret_cast<const T*>(S.ops) : reinterpret_cast<const T*>(S.opsf);
          for (int64_t lb = tk.b; lb < e1; ++lb)
            translate_tile<T, MT>(static_cast<T*>(S.data), S.box_stride, cm, S.Q, S.KS, P.tgt_box, P.src_ptr,
                                  P.src_box, P.src_op, ops, int(lb % P.ntgt), lb / P.ntgt);
          break;
        }
        case kTL2P:
          for (int g = tk.a; g < tk.b; ++g) {
            const GemmTile tl = S.t_l2p[g];
            gemm_tile<MODE, true, double>(S.d_l2p[tl.prob], tl.mt, tl.nt, Cg, ldcg, GemmRun{}, sm);
          }
          break;
        case kTReduce: {    // rows [a, b)
          const int64_t n = int64_t(tk.b - tk.a) * S.nocc;
          for (int64_t e = tid; e < n; e += 256)
            reduce_elem(S.KB, S.nocc, S.occ_ptr, S.occ_row, S.K, S.ldk, 0, 0, int(tk.a + e / S.nocc), e % S.nocc);
          break;
        }
        default:
          break;
      }
      __syncthreads();   // shared memory is reused by the block's next task
    }
    grid.sync();
  }
}

// --------------------------------------------------------------------------
// host side
// --------------------------------------------------------------------------
static void build_tasks(BatchPlan& bp) {
  std::vector<BTask> tasks;
  // stages per system
  struct Stage {
    std::vector<BTask> t;
  };
  std::vector<std::vector<Stage>> st(bp.nsys);
  int maxst = 0;
  for (int k = 0; k < bp.nsys; ++k) {
    Tree* t = bp.trees[k];
    DeviceState* ds = t->dev;
    const BSys& S = bp.host_sys[k];
    auto& v = st[k];
    Stage prep;
    for (int o = 0; o < int(t->ops.size()); ++o) prep.t.push_back({kTOpgen, int16_t(k), o, 0});
    if (bp.prec != OCCK_PREC_FP64)
      for (int64_t r = 0; r < S.nbasis; r += kConvertRows)
        prep.t.push_back({kTConvert, int16_t(k), int32_t(r), int32_t(std::min<int64_t>(S.nbasis, r + kConvertRows))});
    v.push_back(prep);
    auto gemm_stage = [&](int16_t type, int n) {
      Stage s;
      for (int g = 0; g < n; g += bp.gemm_group)
        s.t.push_back({type, int16_t(k), g, std::min(n, g + bp.gemm_group)});
      v.push_back(s);
    };
    gemm_stage(kTHalf, ds->n_half);
    gemm_stage(kTOmega, ds->n_omega);
    const int np = int(ds->up.size() + ds->down.size());
    for (int p = 0; p < np; ++p) {
      const BPass& P = bp.host_passes[S.pass0 + p];
      Stage s;
      for (int64_t lb = 0; lb < P.nblocks; lb += bp.trans_group)
        s.t.push_back({kTTrans, int16_t(k), p, int32_t(lb)});
      v.push_back(s);
    }
    gemm_stage(kTL2P, ds->n_l2p);
    Stage red;
    for (int r = 0; r < S.nbasis; r += kReduceRows)
      red.t.push_back({kTReduce, int16_t(k), r, std::min(S.nbasis, r + kReduceRows)});
    v.push_back(red);
    maxst = std::max(maxst, int(v.size()));
  }
  // stage-grouped list: stage s of every system that has one
  std::vector<int32_t> sptr{0};
  for (int s = 0; s < maxst; ++s) {
    for (int k = 0; k < bp.nsys; ++k)
      if (s < int(st[k].size())) tasks.insert(tasks.end(), st[k][s].t.begin(), st[k][s].t.end());
    sptr.push_back(int32_t(tasks.size()));
  }
  bp.ntasks = int(tasks.size());
  bp.nstage = maxst;
  bp.tasks.upload(tasks);
  bp.stage_ptr.upload(sptr);
}

static void prepare(BatchPlan& bp, hipStream_t st) {
  const bool mixed = bp.prec != OCCK_PREC_FP64;
  bp.host_sys.assign(bp.nsys, BSys{});
  bp.ws_gen.assign(size_t(bp.nsys), 0);
  bp.host_passes.clear();
  for (int k = 0; k < bp.nsys; ++k) {
    Tree* t = bp.trees[k];
    if (!t->dev) upload_tree(t);
    DeviceState* ds = t->dev;
    if (mixed) ensure_mixed_operands(t, st);
    const int n = bp.nocc[k];
    setup_workspace(t, n, n, bp.prec);
    if (mixed) ds->Cf.alloc(size_t(t->nbasis) * n);
    bp.ws_gen[size_t(k)] = ds->ws_gen;
    BSys& S = bp.host_sys[k];
    S.d_half = ds->d_half.p;
    S.t_half = ds->t_half.p;
    S.d_omega = ds->d_omega.p;
    S.t_omega = ds->t_omega.p;
    S.d_l2p = ds->d_l2p.p;
    S.t_l2p = ds->t_l2p.p;
    S.Cf = mixed ? ds->Cf.p : nullptr;
    S.data = ds->data.p;
    S.ncol = int64_t(n) * n;
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
    S.pass0 = int(bp.host_passes.size());
    const int64_t nct = (S.ncol + 255) / 256;
    for (const Pass& p : ds->up)
      bp.host_passes.push_back({p.tgt_box.p, p.src_ptr.p, p.src_box.p, p.src_op.p, p.ntgt, 0, nct * p.ntgt});
    for (const Pass& p : ds->down)
      bp.host_passes.push_back({p.tgt_box.p, p.src_ptr.p, p.src_box.p, p.src_op.p, p.ntgt, 0, nct * p.ntgt});
  }
  bp.passes.upload(bp.host_passes);
  bp.sys.upload(bp.host_sys);
  build_tasks(bp);
}

template <int MODE, int MT>
static void launch_coop(BatchPlan& bp, hipStream_t st) {
  auto kern = batch_kernel<MODE, MT>;
  int per_cu = 0;
  HIP_OK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void*>(kern), 256, 0));
  if (per_cu < 1) throw HipError("batch kernel cannot be resident");
  bp.max_blocks_per_cu = per_cu;
  const int grid = bp.ncu * std::min(bp.blocks_per_cu, per_cu);
  const BTask* tasks = bp.tasks.p;
  const int32_t* sptr = bp.stage_ptr.p;
  int nstage = bp.nstage;
  const BSys* sys = bp.sys.p;
  const BPass* passes = bp.passes.p;
  int gg = bp.gemm_group, tg = bp.trans_group;
  void* args[] = {&tasks, &sptr, &nstage, &sys, &passes, &gg, &tg};
  HIP_OK(hipLaunchCooperativeKernel(reinterpret_cast<const void*>(kern), dim3(unsigned(grid)), dim3(256), args, 0,
                                    st));
}

template <int MODE>
static void launch_batch(BatchPlan& bp, hipStream_t st) {
  switch (mtiles_of(bp.Q)) {
    case 1: launch_coop<MODE, 1>(bp, st); break;
    case 2: launch_coop<MODE, 2>(bp, st); break;
    case 3: launch_coop<MODE, 3>(bp, st); break;
    case 4: launch_coop<MODE, 4>(bp, st); break;
    case 5: launch_coop<MODE, 5>(bp, st); break;
    case 6: launch_coop<MODE, 6>(bp, st); break;
    default: throw std::invalid_argument("unsupported Q");
  }
}

static void launch(BatchPlan& bp, hipStream_t st) {
  switch (bp.prec) {
    case OCCK_PREC_FP64: launch_batch<kModeF64>(bp, st); break;
    case OCCK_PREC_FP32: launch_batch<kModeF32>(bp, st); break;
    case OCCK_PREC_BF16X3: launch_batch<kModeBF16x3>(bp, st); break;
    default: launch_batch<kModeBF16x6>(bp, st); break;
  }
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
int32_t batch_create(int nsys, Tree* const* trees, const int32_t* nocc, int prec, void** out) {
  BatchPlan* bp = new BatchPlan();
  try {
    bp->nsys = nsys;
    bp->prec = prec;
    bp->trees.assign(trees, trees + nsys);
    bp->nocc.assign(nocc, nocc + nsys);
    bp->L = trees[0]->L;
    bp->Q = trees[0]->Q;
    int dev = 0;
    HIP_OK(hipGetDevice(&dev));
    hipDeviceProp_t prop;
    HIP_OK(hipGetDeviceProperties(&prop, dev));
    bp->ncu = prop.multiProcessorCount;
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
    if (!ds || ds->ws_jb != bp.nocc[k] || ds->ws_ni != bp.nocc[k] || ds->ws_prec != bp.prec ||
        ds->ws_gen != bp.ws_gen[size_t(k)] || (bp.prec != OCCK_PREC_FP64 && ds->Cf.p != bp.host_sys[k].Cf))
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
  }
  return OCCK_OK;
}

// Times every candidate (blocks per CU, GEMM tiles per task, translation
// column tiles per task) once after a warm-up and keeps the fastest.
int32_t batch_tune(void* plan, const double* const* C, const int64_t* ldc, double* const* K, const int64_t* ldk,
                   void* stream, int32_t* choice) {
  BatchPlan& bp = *static_cast<BatchPlan*>(plan);
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  const int bpc[] = {1, 2, 4};
  const int gg[] = {1, 2};
  const int tg[] = {1, 4};
  double best = 1e300;
  int bb = 2, bg = 1, bt = 1;
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
  bp->magic = 0;
  delete bp;
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
