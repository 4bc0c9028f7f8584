// Far-field Coulomb matrix through the occ-FMM tree (Le & Shiozaki,
// arXiv:1708.05353, Theory section: the Coulomb passage with Eq. 10 and the
// J^ff formula that follows it), for gfx950.
//
// One density column instead of the (i, j) columns of the exchange:
//   jdens   partial density-contracted multipoles of a chunk of a leaf's pairs,
//           O^B_q += sum_{(t,u)} O^{tu,B}_q D_tu
//   jsum    the chunks of each leaf summed in a fixed order
//   jtrans  one launch per level: upward M2M (Eq. 11), then downward, each box
//           taking its parent's local expansion (L2L, Eq. 13) and its
//           interaction list (M2L, Eq. 12, the hierarchical form of Eq. 10)
//   jpair   J_rs = sum_lm O^{rs,B}_lm Mloc^B_lm for every pair of every leaf
//
// The work is a few passes over the pair multipoles (Q values per screened
// pair) and over small per-box vectors: it is bound by HBM bandwidth, not by
// arithmetic, so every kernel is laid out for coalesced streaming reads.
//
// Data layout in HBM (FP64):
//   pm      pair multipoles [pair][q], pairs in leaf order (the q values of a
//           pair contiguous: a wave reads them as one coalesced row)
//   data    Omega of every box on levels lmin..depth (rows 0..nbox-1), then
//           the local expansions Mloc (rows nbox..2 nbox-1), Q values per row
//   ops     translation operators, real form, Q x Q column-major
//   part    per chunk of pairs, the partial density multipoles (Q values)
#include <hip/hip_runtime.h>

#include <algorithm>
#include <new>
#include <stdexcept>
#include <vector>

#include "device.hpp"

namespace occk {

constexpr int kJChunk = 256;   // pairs per chunk (a chunk never spans two leaves)

// ---------------------------------------------------------------------------
// kernels
// ---------------------------------------------------------------------------
// Real-form translation operator (unweighted), column-major: element
// col*Q + row.  FP64 by the recurrences of Eqs. (4a,b), one block per operator.
static __global__ __launch_bounds__(256) void jopgen_kernel(const OpParam* __restrict__ params,
                                                            double* __restrict__ ops, int L, int Q) {
  __shared__ Cplx tab[(2 * kMaxLTree + 1) * (2 * kMaxLTree + 2) / 2];
  const OpParam p = params[blockIdx.x];
  if (threadIdx.x == 0) {
    if (p.type == kOpM2L) irregular_table(2 * L, p.d, tab);
    else regular_table(L, p.d, tab);
  }
  __syncthreads();
  double* out = ops + int64_t(blockIdx.x) * Q * Q;
  for (int e = threadIdx.x; e < Q * Q; e += blockDim.x) out[e] = real_entry(p.type, tab, e % Q, e / Q);
}

// part[c][q] = sum over the pairs k of chunk c of pm[k][q] D[r_k, s_k]; one
// thread per component q, the chunk's density elements staged in LDS.
static __global__ __launch_bounds__(256) void jdens_kernel(const double* __restrict__ pm,
                                                           const int32_t* __restrict__ pr,
                                                           const int32_t* __restrict__ ps,
                                                           const int32_t* __restrict__ chunk0,
                                                           const double* __restrict__ D, int64_t ldd, int Q,
                                                           double* __restrict__ part) {
  __shared__ double dk[kJChunk];
  const int c = blockIdx.x;
  const int k0 = chunk0[c], n = chunk0[c + 1] - k0;
  for (int k = threadIdx.x; k < n; k += blockDim.x) dk[k] = D[int64_t(pr[k0 + k]) * ldd + ps[k0 + k]];
  __syncthreads();
  for (int q = threadIdx.x; q < Q; q += blockDim.x) {
    const double* p = pm + int64_t(k0) * Q + q;
    double acc = 0.0;
    for (int k = 0; k < n; ++k) acc = fma(p[int64_t(k) * Q], dk[k], acc);
    part[int64_t(c) * Q + q] = acc;
  }
}

// Omega of each leaf: its chunks' partial sums in chunk order (deterministic).
static __global__ __launch_bounds__(256) void jsum_kernel(const double* __restrict__ part,
                                                          const int32_t* __restrict__ leaf_chunk0,
                                                          const int32_t* __restrict__ leaf_slot, int Q,
                                                          double* __restrict__ data) {
  const int b = blockIdx.x;
  const int c0 = leaf_chunk0[b], c1 = leaf_chunk0[b + 1];
  for (int q = threadIdx.x; q < Q; q += blockDim.x) {
    double acc = 0.0;
    for (int c = c0; c < c1; ++c) acc += part[int64_t(c) * Q + q];
    data[int64_t(leaf_slot[b]) * Q + q] = acc;
  }
}

// One level of translations: row tgt[t] of data = sum over the target's
// sources e of T_{sop[e]} (row sidx[e] of data).  One block per target, one
// thread per output component; each source row is staged in LDS.
static __global__ __launch_bounds__(256) void jtrans_kernel(double* __restrict__ data,
                                                            const int32_t* __restrict__ tgt,
                                                            const int32_t* __restrict__ sptr,
                                                            const int32_t* __restrict__ sidx,
                                                            const int32_t* __restrict__ sop,
                                                            const double* __restrict__ ops, int Q) {
  __shared__ double xs[256];
  const int t = blockIdx.x, q = threadIdx.x;
  double acc = 0.0;
  for (int e = sptr[t]; e < sptr[t + 1]; ++e) {
    __syncthreads();   // the previous source row has been used by every thread
    if (q < Q) xs[q] = data[int64_t(sidx[e]) * Q + q];
    __syncthreads();
    if (q < Q) {
      const double* T = ops + int64_t(sop[e]) * Q * Q + q;
      for (int c = 0; c < Q; ++c) acc = fma(T[int64_t(c) * Q], xs[c], acc);
    }
  }
  if (q < Q) data[int64_t(tgt[t]) * Q + q] = acc;
}

// Real inner product weights of sum_{m=-l..l} O_lm Mloc_lm over the m >= 0
// components: 1 for (l, 0), 2 for Re, -2 for Im.
__device__ inline double jweight(int q) {
  int l, m, p;
  decode(q, l, m, p);
  if (m == 0) return 1.0;
  return p == 0 ? 2.0 : -2.0;
}

__device__ inline double wave_sum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// J[r_k, s_k] (+)= sum_q w_q pm[k][q] Mloc_q of the pair's leaf; one wave per
// pair at a time (a coalesced row of Q values, then a fixed-order butterfly sum).
static __global__ __launch_bounds__(256) void jpair_kernel(const double* __restrict__ pm,
                                                           const int32_t* __restrict__ pr,
                                                           const int32_t* __restrict__ ps,
                                                           const int32_t* __restrict__ chunk0,
                                                           const int32_t* __restrict__ chunk_row,
                                                           const double* __restrict__ data, int Q,
                                                           double* __restrict__ J, int64_t ldj, int accumulate) {
  __shared__ double wm[256];
  const int c = blockIdx.x;
  const int k0 = chunk0[c], k1 = chunk0[c + 1];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  if (tid < Q) wm[tid] = jweight(tid) * data[int64_t(chunk_row[c]) * Q + tid];
  __syncthreads();
  for (int k = k0 + wave; k < k1; k += 4) {
    const double* p = pm + int64_t(k) * Q;
    double v = 0.0;
    for (int q = lane; q < Q; q += 64) v = fma(p[q], wm[q], v);
    v = wave_sum(v);
    if (lane == 0) {
      double* dst = J + int64_t(pr[k]) * ldj + ps[k];
      *dst = accumulate ? *dst + v : v;
    }
  }
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
struct JPass {   // one level of translations, CSR over its targets
  int ntgt = 0;
  DevBuf<int32_t> tgt, sptr, sidx, sop;
};

struct JState {
  int device = -1, Q = 0, nbox = 0, nchunk = 0, nleaf = 0, nops = 0;
  DevBuf<double> pm, ops, data, part;
  DevBuf<OpParam> opparam;
  DevBuf<int32_t> pr, ps, chunk0, chunk_row, leaf_chunk0, leaf_slot;
  std::vector<JPass> up, down;   // up: levels depth-1 .. lmin; down: lmin .. depth
  size_t bytes = 0;
};

void jstate_free(Tree* t) {
  delete t->jdev;   // the DevBufs free their memory
  t->jdev = nullptr;
}

static void jpass_upload(JPass& ps, const std::vector<int32_t>& tg, const std::vector<int32_t>& sp,
                         const std::vector<int32_t>& si, const std::vector<int32_t>& so) {
  ps.ntgt = int(tg.size());
  ps.tgt.upload(tg);
  ps.sptr.upload(sp);
  ps.sidx.upload(si);
  ps.sop.upload(so);
}

// Device bytes the Coulomb path needs for tree t (checked before any HIP call).
static size_t jstate_need(const Tree* t, int64_t* nchunk_out) {
  const int Q = t->Q, D = t->params.depth;
  int64_t nchunk = 0, nbox = 0;
  for (const auto& lp : t->leaf_pairs) nchunk += (int64_t(lp.size()) + kJChunk - 1) / kJChunk;
  for (int lev = t->lmin; lev <= D; ++lev) nbox += int64_t(t->boxes[lev].size());
  if (nchunk_out) *nchunk_out = nchunk;
  return (size_t(t->pairs.size()) * Q + size_t(t->ops.size()) * Q * Q + size_t(2 * nbox) * Q +
          size_t(nchunk) * Q) * 8 + (size_t(t->pairs.size()) * 2 + size_t(nchunk) * 2) * 4;
}

static void jstate_upload(Tree* t) {
  int64_t nchunk = 0;
  const size_t need = jstate_need(t, &nchunk);
  if (need > device_cap()) throw std::bad_alloc();
  JState* js = new JState();
  try {
    HIP_OK(hipGetDevice(&js->device));
    const int Q = t->Q, D = t->params.depth, lmin = t->lmin, nl = t->nleaf();
    js->Q = Q;
    js->nleaf = nl;
    js->nchunk = int(nchunk);
    std::vector<int32_t> slot0(size_t(D + 1), 0);
    int nbox = 0;
    for (int lev = lmin; lev <= D; ++lev) {
      slot0[size_t(lev)] = nbox;
      nbox += int(t->boxes[lev].size());
    }
    js->nbox = nbox;
    // pairs in leaf order, their multipoles, chunks
    std::vector<int32_t> pr, ps, chunk0, chunk_row, leaf_chunk0{0}, leaf_slot;
    pr.reserve(t->pairs.size());
    ps.reserve(t->pairs.size());
    js->pm.alloc(t->pairs.size() * size_t(Q));
    std::vector<double> buf;
    int64_t k = 0;
    for (int b = 0; b < nl; ++b) {
      const auto& lp = t->leaf_pairs[size_t(b)];
      buf.resize(lp.size() * size_t(Q));
      leaf_pair_multipoles(*t, b, buf.data());
      HIP_OK(hipMemcpy(js->pm.p + k * Q, buf.data(), buf.size() * 8, hipMemcpyHostToDevice));
      for (size_t a = 0; a < lp.size(); ++a) {
        if (a % kJChunk == 0) {
          chunk0.push_back(int32_t(k + int64_t(a)));
          chunk_row.push_back(nbox + slot0[size_t(D)] + b);   // the leaf's Mloc row
        }
        pr.push_back(t->pairs[size_t(lp[a])].r);
        ps.push_back(t->pairs[size_t(lp[a])].s);
      }
      k += int64_t(lp.size());
      leaf_chunk0.push_back(int32_t(chunk0.size()));
      leaf_slot.push_back(slot0[size_t(D)] + b);
    }
    chunk0.push_back(int32_t(k));
    js->pr.upload(pr);
    js->ps.upload(ps);
    js->chunk0.upload(chunk0);
    js->chunk_row.upload(chunk_row);
    js->leaf_chunk0.upload(leaf_chunk0);
    js->leaf_slot.upload(leaf_slot);
    // operators (the tree's displacements, unweighted)
    std::vector<OpParam> op(t->ops.size());
    for (size_t e = 0; e < op.size(); ++e) {
      op[e].type = t->ops[e].type;
      op[e].weighted = 0;
      for (int d = 0; d < 3; ++d) op[e].d[d] = t->ops[e].d[d];
    }
    js->nops = int(op.size());
    js->opparam.upload(op);
    js->ops.alloc(op.size() * size_t(Q) * Q);
    js->data.alloc(size_t(2 * nbox) * Q);
    js->part.alloc(size_t(nchunk) * Q);
    // upward passes: parents at lev take their children's Omega (M2M)
    for (int lev = D - 1; lev >= lmin; --lev) {
      const auto& par = t->boxes[lev];
      std::vector<std::vector<std::pair<int32_t, int32_t>>> lists(par.size());
      for (int32_t c = 0; c < int32_t(t->boxes[lev + 1].size()); ++c) {
        const auto& cc = t->boxes[lev + 1][size_t(c)];
        const int oct = (cc[0] & 1) | ((cc[1] & 1) << 1) | ((cc[2] & 1) << 2);
        lists[size_t(t->parent(lev + 1, c))].push_back({slot0[size_t(lev + 1)] + c, t->op_up[(lev + 1) * 8 + oct]});
      }
      std::vector<int32_t> tg, sp{0}, si, so;
      for (size_t p = 0; p < par.size(); ++p) {
        tg.push_back(slot0[size_t(lev)] + int32_t(p));
        for (const auto& e : lists[p]) { si.push_back(e.first); so.push_back(e.second); }
        sp.push_back(int32_t(si.size()));
      }
      js->up.emplace_back();
      jpass_upload(js->up.back(), tg, sp, si, so);
    }
    // downward passes: the parent's Mloc (L2L) first, then the interaction list's Omega (M2L)
    for (int lev = lmin; lev <= D; ++lev) {
      const auto& bx = t->boxes[lev];
      std::vector<int32_t> tg, sp{0}, si, so;
      for (int32_t b = 0; b < int32_t(bx.size()); ++b) {
        tg.push_back(nbox + slot0[size_t(lev)] + b);
        if (lev > lmin) {
          const auto& c = bx[size_t(b)];
          const int oct = (c[0] & 1) | ((c[1] & 1) << 1) | ((c[2] & 1) << 2);
          si.push_back(nbox + slot0[size_t(lev - 1)] + t->parent(lev, b));
          so.push_back(t->op_down[lev * 8 + oct]);
        }
        for (int32_t e = t->il_ptr[lev][size_t(b)]; e < t->il_ptr[lev][size_t(b) + 1]; ++e) {
          const int32_t b2 = t->il_idx[lev][size_t(e)];
          const auto& c2 = bx[size_t(b2)];
          const int64_t key = coord_key(bx[size_t(b)][0] - c2[0] + 64, bx[size_t(b)][1] - c2[1] + 64,
                                        bx[size_t(b)][2] - c2[2] + 64);
          si.push_back(slot0[size_t(lev)] + b2);
          so.push_back(t->op_m2l[lev].at(key));
        }
        sp.push_back(int32_t(si.size()));
      }
      js->down.emplace_back();
      jpass_upload(js->down.back(), tg, sp, si, so);
    }
    js->bytes = need;
  } catch (...) {
    delete js;
    throw;
  }
  t->jdev = js;
}

static inline unsigned jthreads(int Q) { return unsigned(std::min(256, (Q + 63) / 64 * 64)); }

int32_t far_J(Tree* t, const double* Dm, int64_t ldd, double* J, int64_t ldj, int32_t accumulate, void* stream) {
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  const int n = t->nbasis;
  try {
    if (t->lmin < 0) {   // no far field
      if (!accumulate)
        hipLaunchKernelGGL(zero_cols_kernel, dim3(unsigned((n + 255) / 256), unsigned(n)), dim3(256), 0, st, J, ldj,
                           0, int64_t(n));
      HIP_OK(hipGetLastError());
      return OCCK_OK;
    }
    if (!t->jdev) jstate_upload(t);
    JState* js = t->jdev;
    const int Q = js->Q;
    const unsigned nt = jthreads(Q);
    hipLaunchKernelGGL(jopgen_kernel, dim3(unsigned(js->nops)), dim3(256), 0, st, js->opparam.p, js->ops.p, t->L, Q);
    hipLaunchKernelGGL(jdens_kernel, dim3(unsigned(js->nchunk)), dim3(nt), 0, st, js->pm.p, js->pr.p, js->ps.p,
                       js->chunk0.p, Dm, ldd, Q, js->part.p);
    hipLaunchKernelGGL(jsum_kernel, dim3(unsigned(js->nleaf)), dim3(nt), 0, st, js->part.p, js->leaf_chunk0.p,
                       js->leaf_slot.p, Q, js->data.p);
    for (const JPass& ps : js->up)
      hipLaunchKernelGGL(jtrans_kernel, dim3(unsigned(ps.ntgt)), dim3(nt), 0, st, js->data.p, ps.tgt.p, ps.sptr.p,
                         ps.sidx.p, ps.sop.p, js->ops.p, Q);
    for (const JPass& ps : js->down)
      hipLaunchKernelGGL(jtrans_kernel, dim3(unsigned(ps.ntgt)), dim3(nt), 0, st, js->data.p, ps.tgt.p, ps.sptr.p,
                         ps.sidx.p, ps.sop.p, js->ops.p, Q);
    if (!accumulate)
      hipLaunchKernelGGL(zero_cols_kernel, dim3(unsigned((n + 255) / 256), unsigned(n)), dim3(256), 0, st, J, ldj, 0,
                         int64_t(n));
    hipLaunchKernelGGL(jpair_kernel, dim3(unsigned(js->nchunk)), dim3(256), 0, st, js->pm.p, js->pr.p, js->ps.p,
                       js->chunk0.p, js->chunk_row.p, js->data.p, Q, J, ldj, accumulate);
    HIP_OK(hipGetLastError());
  } catch (const HipError& e) {
    set_error(e.what());
    return OCCK_EHIP;
  } catch (const std::bad_alloc&) {
    set_error("occk_far_J: device memory exceeds OCCK_MAX_DEVICE_BYTES or allocation failed");
    return OCCK_ENOMEM;
  }
  return OCCK_OK;
}

}  // namespace occk
