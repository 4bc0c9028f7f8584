// GPU hot path of the far-field occupied exchange (occ-FMM-K, Le & Shiozaki,
// arXiv:1708.05353, Theory section, Eqs. 15-18) for gfx950.
//
// Per call (all on the caller's stream):
//   opgen      FP64 translation operators by recurrence (Eqs. 4, 11-13)
//   per batch of occupied j columns (the paper distributes Step 2 by j batches):
//     half     H^B_q = O^B_q C_B[:, J]                      Eq. (15a)   MFMA GEMM
//     omega    Omega^B[(q,j), i] = sum_t H^B_q[t, j] C[t, i]  Eq. (15b)   MFMA GEMM
//     up       Omega^p = sum_c T_up(c) Omega^c              Eq. (17a)   translation
//     down     Mloc^b = T_down Mloc^parent + sum_IL T Omega   Eq. (17b,c) translation
//     l2p      KB^B[r, i] += sum_(q,j) H^B[r,(q,j)] Mloc^B[(q,j), i]   Eq. (18)
//   reduce     K[r, i] = sum over the leaves holding r of KB       (deterministic)
//
// Data layout in HBM (FP64): the box data of one batch is Q rows x ncol
// columns per box, column c = j_local * n_i + i_local, row q = real
// component.  Omega and Mloc of all boxes on levels lmin..depth live in one
// buffer (Omega boxes first, then Mloc boxes).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <functional>
#include <map>
#include <mutex>
#include <stdexcept>
#include <tuple>
#include <string>
#include <type_traits>
#include <vector>


#include "device.hpp"

namespace occk {

size_t device_cap() {
  const char* s = std::getenv("OCCK_MAX_DEVICE_BYTES");
  if (s && *s) return size_t(std::strtoull(s, nullptr, 10));
  return size_t(96) << 30;
}

static void free_state(DeviceState* ds);

static void upload_tree_into(Tree* t, DeviceState* ds);


// The walks pay off where a block's subtree is a long chain of cheap steps
// (binary splits, short interaction lists: the chain-like trees); on 2-D
// and 3-D trees, with up to 8 children and tens of interaction-list
// sources per box, the level-by-level passes keep more waves busy and are
// faster.  Both walks are used when the boxes above the leaves have at
// most 2 children on average and the interaction lists at most 8 sources.
bool walk_tree(const Tree* t) {
  const int lmin = t->lmin, D = t->params.depth;
  if (lmin < 0) return false;
  int64_t n_above = 0, n_kids = 0, n_tgt = 0, n_src = 0;
  for (int lev = lmin; lev < D; ++lev) {
    n_above += int64_t(t->boxes[lev].size());
    n_kids += int64_t(t->boxes[lev + 1].size());
  }
  for (int lev = lmin; lev <= D; ++lev) {
    n_tgt += int64_t(t->boxes[lev].size());
    n_src += int64_t(t->il_idx[lev].size());
  }
  return t->Q <= 9 && n_kids <= 2 * n_above && n_src <= 8 * n_tgt;
}

void upload_tree(Tree* t) {
  if (t->lmin < 0) throw std::invalid_argument("upload_tree: the tree has no far field");
  DeviceState* ds = new DeviceState();
  try {
    upload_tree_into(t, ds);
  } catch (...) {
    free_state(ds);
    throw;
  }
  t->dev = ds;
}

// One level of translations on the host: targets, CSR of sources, operators
// (box slots as in the passes: upward Omega slots, downward Mloc rows).
struct HostLevel {
  std::vector<int32_t> tgt, ptr, src, op;
};

// Stencil tables of tree_chain_kernel when the tree is a chain in its
// sense: the boxes of every level one unbroken row along x at equal y and z
// (x = x0 + b for box b); every box above the leaves lists its children
// present in increasing x, with one operator per child x parity; every box
// below the first level lists its parent first, with one operator per x
// parity; and every interaction list is the in-range part of one stencil per
// level and x parity (the displacements of that parity's lists, in
// increasing order, one operator each).  Leaves ds->chain_nlev at 0
// otherwise.
static void build_chain(const Tree* t, DeviceState* ds, const std::vector<HostLevel>& hup,
                        const std::vector<HostLevel>& hdn, const std::vector<int32_t>& slot0) {
  const int lmin = t->lmin, D = t->params.depth;
  const int32_t nbox = ds->nbox;
  const int nlev = D - lmin + 1;
  std::vector<ChainLevel> lv(static_cast<size_t>(nlev));
  for (int li = 0; li < nlev; ++li) {
    const int lev = lmin + li;
    const auto& bx = t->boxes[size_t(lev)];
    ChainLevel& L = lv[size_t(li)];
    L = ChainLevel{};
    const HostLevel& h = hdn[size_t(li)];
    L.n = int32_t(bx.size());
    L.slot0 = slot0[size_t(lev)];
    if (L.n == 0 || int32_t(h.tgt.size()) != L.n) return;
    L.x0 = bx[0][0];
    for (int32_t b = 0; b < L.n; ++b)
      if (bx[size_t(b)][0] != L.x0 + b || bx[size_t(b)][1] != bx[0][1] || bx[size_t(b)][2] != bx[0][2]) return;
    // the stencil of each x parity: every displacement of that parity's
    // interaction lists, in increasing order, with its one operator
    std::map<int32_t, int32_t> sten[2];
    const int first = li > 0 ? 1 : 0;   // entry 0 is the parent's local expansion below the first level
    for (int32_t b = 0; b < L.n; ++b) {
      if (h.tgt[size_t(b)] != nbox + L.slot0 + b) return;
      const int par = (L.x0 + b) & 1;
      if (h.ptr[size_t(b) + 1] - h.ptr[size_t(b)] < first) return;
      for (int32_t e = h.ptr[size_t(b)] + first; e < h.ptr[size_t(b) + 1]; ++e) {
        const int32_t d = h.src[size_t(e)] - (L.slot0 + b);
        auto it = sten[par].emplace(d, h.op[size_t(e)]).first;
        if (it->second != h.op[size_t(e)]) return;
      }
    }
    for (int par = 0; par < 2; ++par) {
      L.dn_op[par] = -1;
      if (sten[par].size() > size_t(kChainStencil)) return;
      L.ne[par] = int32_t(sten[par].size());
      int e = 0;
      for (const auto& kv : sten[par]) {
        L.d[par][e] = kv.first;
        L.op[par][e] = kv.second;
        ++e;
      }
    }
    // every box: parent, then the in-range part of its parity's stencil
    for (int32_t b = 0; b < L.n; ++b) {
      const int par = (L.x0 + b) & 1;
      int32_t e = h.ptr[size_t(b)];
      if (li > 0) {
        const ChainLevel& P = lv[size_t(li - 1)];
        const int32_t pb = ((L.x0 + b) >> 1) - P.x0;
        if (pb < 0 || pb >= P.n || h.src[size_t(e)] != nbox + P.slot0 + pb) return;
        if (L.dn_op[par] < 0) L.dn_op[par] = h.op[size_t(e)];
        if (h.op[size_t(e)] != L.dn_op[par]) return;
        ++e;
      }
      for (int k = 0; k < L.ne[par]; ++k) {
        const int32_t s = b + L.d[par][k];
        if (s < 0 || s >= L.n) continue;
        if (e >= h.ptr[size_t(b) + 1] || h.src[size_t(e)] != L.slot0 + s || h.op[size_t(e)] != L.op[par][k]) return;
        ++e;
      }
      if (e != h.ptr[size_t(b) + 1]) return;
    }
  }
  // upward: hup[k] holds level D - 1 - k as targets; children present in increasing x
  for (int li = 0; li + 1 < nlev; ++li) {
    const HostLevel& h = hup[size_t(D - 1 - (lmin + li))];
    ChainLevel& L = lv[size_t(li)];
    const ChainLevel& Cl = lv[size_t(li + 1)];
    if (int32_t(h.tgt.size()) != L.n) return;
    L.up_op[0] = L.up_op[1] = -1;
    for (int32_t p = 0; p < L.n; ++p) {
      if (h.tgt[size_t(p)] != L.slot0 + p) return;
      int32_t e = h.ptr[size_t(p)];
      for (int k = 0; k < 2; ++k) {
        const int32_t ci = 2 * (L.x0 + p) + k - Cl.x0;
        if (ci < 0 || ci >= Cl.n) continue;
        if (e >= h.ptr[size_t(p) + 1] || h.src[size_t(e)] != Cl.slot0 + ci) return;
        if (L.up_op[k] < 0) L.up_op[k] = h.op[size_t(e)];
        if (h.op[size_t(e)] != L.up_op[k]) return;
        ++e;
      }
      if (e != h.ptr[size_t(p) + 1]) return;
    }
  }
  ds->chain.upload(lv);
  ds->chain_nlev = nlev;
  ds->chain_nbelow = nlev > 1 ? lv[size_t(nlev - 2)].n : 0;
}

static void upload_tree_into(Tree* t, DeviceState* ds) {
  HIP_OK(hipGetDevice(&ds->device));
  const int D = t->params.depth, Q = t->Q, nl = t->nleaf();
  // leaf blocks
  int64_t tot = 0, ftot = 0;
  ds->O_off.resize(nl + 1);
  ds->f_off.resize(nl + 1);
  for (int b = 0; b < nl; ++b) {
    const int64_t nb = int64_t(t->leaf_funcs[b].size());
    ds->O_off[b] = tot;
    ds->f_off[b] = ftot;
    tot += int64_t(Q) * nb * nb;
    ftot += nb;
  }
  ds->O_off[nl] = tot;
  ds->f_off[nl] = ftot;
  if (size_t(tot) * 8 > device_cap()) throw std::bad_alloc();
  ds->O.alloc(size_t(tot));
  {
    std::vector<double> buf;
    for (int b = 0; b < nl; ++b) {
      const int64_t n = ds->O_off[b + 1] - ds->O_off[b];
      buf.resize(size_t(n));
      leaf_multipoles(*t, b, buf.data());
      HIP_OK(hipMemcpy(ds->O.p + ds->O_off[b], buf.data(), size_t(n) * 8, hipMemcpyHostToDevice));
    }
  }
  std::vector<int32_t> fl;
  fl.reserve(size_t(ftot));
  for (int b = 0; b < nl; ++b) fl.insert(fl.end(), t->leaf_funcs[b].begin(), t->leaf_funcs[b].end());
  ds->funcs.upload(fl);
  // operators
  std::vector<OpParam> op(t->ops.size());
  for (size_t k = 0; k < op.size(); ++k) {
    op[k].type = t->ops[k].type;
    op[k].weighted = t->ops[k].weighted;
    for (int d = 0; d < 3; ++d) op[k].d[d] = t->ops[k].d[d];
  }
  ds->opparam.upload(op);
  // structural zeros of the translation operators: every displacement on
  // the x axis (1) or in the xy plane (2), else none (0)
  bool xaxis = true, xyplane = true;
  for (const OpParam& o : op) {
    xaxis = xaxis && o.d[1] == 0.0 && o.d[2] == 0.0;
    xyplane = xyplane && o.d[2] == 0.0;
  }
  ds->op_sym = xaxis ? 1 : xyplane ? 2 : 0;
  if (ds->op_sym != 0 && Q > 9) {   // MFMA translations: components grouped by class (stable in q)
    std::vector<int32_t> perm(static_cast<size_t>(Q));
    for (int q = 0; q < Q; ++q) perm[size_t(q)] = q;
    std::stable_sort(perm.begin(), perm.end(), [&](int32_t a, int32_t b) {
      return real_class(a, ds->op_sym) < real_class(b, ds->op_sym);
    });
    std::vector<int8_t> cls(static_cast<size_t>(Q));
    for (int k = 0; k < Q; ++k) cls[size_t(k)] = int8_t(real_class(perm[size_t(k)], ds->op_sym));
    ds->perm.upload(perm);
    ds->pcls.upload(cls);
    ds->ops_perm.alloc(op.size() * size_t(opsize_of(Q)));
  }
  ds->ops.alloc(op.size() * size_t(opsize_of(Q)));
  // box slots on levels lmin..D
  const int lmin = t->lmin;
  std::vector<int32_t> slot0(D + 1, 0);
  int nbox = 0;
  for (int lev = lmin; lev <= D; ++lev) {
    slot0[lev] = nbox;
    nbox += int(t->boxes[lev].size());
  }
  ds->nbox = nbox;
  ds->leaf_box.resize(nl);
  for (int b = 0; b < nl; ++b) ds->leaf_box[b] = slot0[D] + b;
  std::vector<HostLevel> hup, hdn;   // host copies for the in-LDS tree programs
  // upward passes: targets at lev (parents), sources children at lev+1 (M2M)
  for (int lev = D - 1; lev >= lmin; --lev) {
    const auto& par = t->boxes[lev];
    std::vector<std::vector<std::pair<int32_t, int32_t>>> lists(par.size());
    for (int32_t c = 0; c < int32_t(t->boxes[lev + 1].size()); ++c) {
      const auto& cc = t->boxes[lev + 1][c];
      const int oct = (cc[0] & 1) | ((cc[1] & 1) << 1) | ((cc[2] & 1) << 2);
      const int32_t p = t->parent(lev + 1, c);
      lists[p].push_back({slot0[lev + 1] + c, t->op_up[(lev + 1) * 8 + oct]});
    }
    Pass ps;
    std::vector<int32_t> tb, sp{0}, sb, so;
    for (size_t p = 0; p < par.size(); ++p) {
      tb.push_back(slot0[lev] + int32_t(p));
      for (auto& e : lists[p]) { sb.push_back(e.first); so.push_back(e.second); }
      sp.push_back(int32_t(sb.size()));
    }
    ps.ntgt = int(par.size());
    ps.nent = int(sb.size());
    ps.host_op = so;
    hup.push_back({tb, sp, sb, so});
    ps.tgt_box.upload(tb);
    ps.src_ptr.upload(sp);
    ps.src_box.upload(sb);
    ps.src_op.upload(so);
    ds->up.push_back(std::move(ps));
  }
  // children of every box above the leaves, in the order of the upward
  // passes' source lists, with their M2M operators
  std::vector<std::vector<std::vector<std::pair<int32_t, int32_t>>>> kids(static_cast<size_t>(D + 1));
  for (int lev = lmin; lev < D; ++lev) {
    kids[size_t(lev)].resize(t->boxes[lev].size());
    for (int32_t c = 0; c < int32_t(t->boxes[lev + 1].size()); ++c) {
      const auto& cc = t->boxes[lev + 1][c];
      const int oct = (cc[0] & 1) | ((cc[1] & 1) << 1) | ((cc[2] & 1) << 2);
      kids[size_t(lev)][size_t(t->parent(lev + 1, c))].push_back({c, t->op_up[(lev + 1) * 8 + oct]});
    }
  }
  const bool walks = walk_tree(t);
  // the upward walk: post-order program of every subtree below a box of
  // level lr = max(lmin, D - kUpWalkLevels); the levels above lr keep their
  // level-by-level passes, which read the walk's level-lr multipoles
  if (walks && D - lmin >= 1) {
    const int lr = std::max(lmin, D - kUpWalkLevels);
    std::vector<WalkStep> prog;
    std::vector<int32_t> pptr{0};
    std::function<void(int, int32_t)> emit = [&](int lev, int32_t p) {
      for (const auto& kc : kids[size_t(lev)][size_t(p)]) {
        if (lev + 1 == D) {
          prog.push_back({UP_LEAF, lev - lr, slot0[D] + kc.first, kc.second});
        } else {
          emit(lev + 1, kc.first);
          prog.push_back({UP_CLOSE, lev + 1 - lr, slot0[lev + 1] + kc.first, kc.second});
        }
      }
    };
    for (int32_t r = 0; r < int32_t(t->boxes[lr].size()); ++r) {
      emit(lr, r);
      prog.push_back({UP_CLOSE, 0, slot0[lr] + r, -1});
      pptr.push_back(int32_t(prog.size()));
    }
    ds->upw_prog.upload(prog);
    ds->upw_ptr.upload(pptr);
    ds->upw_nroots = int(t->boxes[lr].size());
    ds->upw_nlv = D - lr;
    ds->upw_lroot = lr;
  }
  // downward passes: Mloc targets at lev; sources = parent Mloc (L2L) + IL Omega (M2L)
  std::vector<std::vector<int32_t>> dn_ptr, dn_box;   // host CSR of each downward level
  for (int lev = lmin; lev <= D; ++lev) {
    const auto& bx = t->boxes[lev];
    Pass ps;
    std::vector<int32_t> tb, sp{0}, sb, so;
    for (int32_t b = 0; b < int32_t(bx.size()); ++b) {
      tb.push_back(nbox + slot0[lev] + b);
      if (lev > lmin) {
        const int oct = (bx[b][0] & 1) | ((bx[b][1] & 1) << 1) | ((bx[b][2] & 1) << 2);
        sb.push_back(nbox + slot0[lev - 1] + t->parent(lev, b));
        so.push_back(t->op_down[lev * 8 + oct]);
      }
      for (int32_t e = t->il_ptr[lev][b]; e < t->il_ptr[lev][b + 1]; ++e) {
        const int32_t b2 = t->il_idx[lev][e];
        const auto& c2 = bx[b2];
        const int64_t key = coord_key(bx[b][0] - c2[0] + 64, bx[b][1] - c2[1] + 64, bx[b][2] - c2[2] + 64);
        sb.push_back(slot0[lev] + b2);
        so.push_back(t->op_m2l[lev].at(key));
      }
      sp.push_back(int32_t(sb.size()));
    }
    ps.ntgt = int(bx.size());
    ps.nent = int(sb.size());
    ps.host_op = so;
    dn_ptr.push_back(sp);
    dn_box.push_back(sb);
    hdn.push_back({tb, sp, sb, so});
    for (int32_t b = 0; b < ps.ntgt; ++b)
      for (int32_t e = sp[b]; e < sp[b + 1]; ++e) ps.host_tgt.push_back(b);
    ps.ent_tgt.upload(ps.host_tgt);
    ps.tgt_box.upload(tb);
    ps.src_ptr.upload(sp);
    ps.src_box.upload(sb);
    ps.src_op.upload(so);
    ds->down.push_back(std::move(ps));
  }
  // the downward walk: pre-order program of every subtree below a box of
  // level lr = max(lmin, D + 1 - kDownWalkLevels); each box's terms in the
  // order of its downward-pass source list.  A walk root reads its parent's
  // local expansion (written by the level-by-level pass of level lr - 1)
  // like any source; below it the parent term comes from the registers.
  if (walks) {
    const int lr = std::max(lmin, D + 1 - kDownWalkLevels);
    std::vector<WalkStep> prog;
    std::vector<int32_t> pptr{0};
    std::function<void(int, int32_t)> visit = [&](int lev, int32_t b) {
      const int lp = lev - lmin, li = lev - lr;   // pass index, accumulator level
      const Pass& ps = ds->down[size_t(lp)];
      int32_t e = dn_ptr[size_t(lp)][size_t(b)];
      const int32_t e1 = dn_ptr[size_t(lp)][size_t(b) + 1];
      if (lev > lr) {   // the parent term (L2L) comes first, from the parent level's accumulator
        prog.push_back({DN_BEGIN, li, 0, ps.host_op[size_t(e)]});
        ++e;
      } else {
        prog.push_back({DN_BEGIN, li, 0, -1});
      }
      for (; e < e1; ++e) prog.push_back({DN_SRC, li, dn_box[size_t(lp)][size_t(e)], ps.host_op[size_t(e)]});
      if (lev == D) {
        prog.push_back({DN_STORE, li, int32_t(nbox) + slot0[D] + b, -1});
      } else {
        for (const auto& kc : kids[size_t(lev)][size_t(b)]) visit(lev + 1, kc.first);
      }
    };
    for (int32_t r = 0; r < int32_t(t->boxes[lr].size()); ++r) {
      visit(lr, r);
      pptr.push_back(int32_t(prog.size()));
    }
    ds->dnw_prog.upload(prog);
    ds->dnw_ptr.upload(pptr);
    ds->dnw_nroots = int(t->boxes[lr].size());
    ds->dnw_nlv = D - lr + 1;
    ds->dnw_lroot = lr;
  }
  if (Q == 9 && ds->op_sym == 1) {
    build_chain(t, ds, hup, hdn, slot0);
    int64_t off = 0;
    for (int cl = 0; cl < (ds->op_sym == 1 ? 4 : 2); ++cl) {
      ds->ops_cls_off[cl] = off;
      const int n = class_size(Q, ds->op_sym, cl);
      off += int64_t(t->ops.size()) * n * n;
    }
    ds->ops_cls.alloc(size_t(off));
  }
  // reduction lists: function r -> rows of KB (leaf order, then local order)
  std::vector<std::vector<int32_t>> occ(t->nbasis);
  for (int b = 0; b < nl; ++b)
    for (size_t a = 0; a < t->leaf_funcs[b].size(); ++a)
      occ[t->leaf_funcs[b][a]].push_back(int32_t(ds->f_off[b] + int64_t(a)));
  std::vector<int32_t> optr{0}, orow;
  for (int r = 0; r < t->nbasis; ++r) {
    orow.insert(orow.end(), occ[r].begin(), occ[r].end());
    optr.push_back(int32_t(orow.size()));
  }
  ds->occ_ptr.upload(optr);
  ds->occ_row.upload(orow);
  ds->bytes = size_t(tot) * 8;
}

template <class S = GemmSquare>
static void tiles_for(std::vector<GemmTile>& tiles, int prob, int M, int N) {
  for (int mt = 0; mt < (M + S::BM - 1) / S::BM; ++mt)
    for (int nt = 0; nt < (N + S::BN - 1) / S::BN; ++nt) tiles.push_back({prob, mt, nt, 0});
}

// Tile lists for launching the column tiles nt >= 4c of every problem
// (c = 0 .. nch-1; the symmetric schedule skips the columns below the first
// carried one).  List c holds those tiles in the order `key`, problem first,
// so that a problem's tiles are adjacent in the launch and its operand panels
// stay in L2 while they run; the lists are stored one after another and list
// c is [start[c], start[c + 1]).
template <class Key>
static std::vector<int32_t> chunked_tile_lists(std::vector<GemmTile>& tiles, Key key) {
  std::stable_sort(tiles.begin(), tiles.end(), [&](const GemmTile& x, const GemmTile& y) { return key(x) < key(y); });
  int nch = 1;
  for (const GemmTile& x : tiles) nch = std::max(nch, x.nt / 4 + 1);
  std::vector<int32_t> start;
  std::vector<GemmTile> out;
  for (int c = 0; c < nch; ++c) {
    start.push_back(int32_t(out.size()));
    for (const GemmTile& x : tiles)
      if (x.nt >= 4 * c) out.push_back(x);
    if (out.size() > size_t(INT32_MAX)) throw std::invalid_argument("far_K: too many GEMM tiles");
  }
  start.push_back(int32_t(out.size()));
  tiles.swap(out);
  return start;
}

// Launch of tiles [tile0, tile0 + n) of a grouped GEMM (grid padded to a
// multiple of 8 for the XCD-aware order).
static inline unsigned gemm_grid(int n) { return unsigned(((n + 7) / 8) * 8); }

// Device bytes of one workspace shape (box data, H, HT, KB).
// extra_rows: box rows beyond Omega and Mloc (the second leaf Mloc region of
// the two-stream schedule).
static size_t workspace_need(int64_t sum_nb, int Q, int64_t nbox, int jb, int ni, size_t es, bool sym,
                             int64_t extra_rows = 0) {
  const int64_t ncol = int64_t(jb) * ni;
  return size_t(sum_nb) * Q * jb * es + size_t(2 * nbox + extra_rows) * Q * size_t(ncol) * es +
         size_t(sum_nb) * ni * 8 + (sym ? size_t(sum_nb) * Q * ni * es : 0);
}

// Buffers and GEMM descriptors of one workspace shape.  Box data of a batch:
// Q rows x ncol = jb*ni columns per box, column (j, i) at j*ni + i.
//   half   H^B[t][q][j] = sum_s O^B_q[t, s] C[s, jstart + j]           (ld Q*jb)
//   omega  Omega^B[(q, j), i] = sum_t H^B[t][(q, j)] C[t, i0 + i]
//   l2p    KB[r, i] (+)= sum_(q,j) H^B[r][(q, j)] Mloc^B[(q, j), i]
// symmetric schedule (sym_mode kWsSym, kWsSymHT) in addition:
//   ht     HT^B[q][i][t] = sum_s O^B_q[t, s] C[s, i0 + i]  for every column i
//   l2pt   KB[r, jstart + j] += sum_q sum_(i >= koff) HT^B[q][i][r] Mloc^B[(q, j), i]
// kWsSymHT reads the batch's H out of HT (no H buffer, no per-batch half):
//   omega  Omega^B[(q, j), i] = sum_t HT^B[q][jstart + j][t] C[t, i0 + i]   (per leaf and q)
//   l2p    KB[r, i] (+)= sum_q sum_j HT^B[q][jstart + j][r] Mloc^B[(q, j), i]   (K segments q)
void setup_workspace(Tree* t, int jb, int ni, int prec, int sym_mode, ScratchArena* arena) {
  DeviceState* ds = t->dev;
  if (!arena && ds->ws_jb == jb && ds->ws_ni == ni && ds->ws_prec == prec && ds->ws_sym == sym_mode) return;
  const bool sym = sym_mode != kWsPlain, from_ht = sym_mode == kWsSymHT;
  const int Q = t->Q, nl = t->nleaf();
  const size_t es = prec == OCCK_PREC_FP64 ? 8 : 4;
  const int64_t sum_nb = ds->f_off[nl];
  const int64_t ncol = int64_t(jb) * ni;
  // the two-stream schedule (occk_far_K, symmetric, downward walks; not in
  // the fixed scratch region) keeps the leaf Mloc of odd batches in nleaf
  // extra box rows
  const bool pipe = from_ht && !arena && ds->dnw_nroots > 0 && ds->upw_nroots > 0;
  const int64_t extra = pipe ? 2 * nl : 0;   // second leaf Mloc rows, then second leaf Omega rows
  const size_t need = workspace_need(sum_nb, Q, ds->nbox, jb, ni, es, sym, extra);
  if (!arena && need + ds->bytes > device_cap()) throw std::bad_alloc();
  // buffers and tables: allocated, or placed in the arena
  auto alloc = [arena](auto& buf, size_t count) {
    if (arena) arena->place(buf, count);
    else buf.alloc(count);
  };
  auto upload = [arena](auto& buf, const auto& v) {
    if (arena) arena->upload(buf, v);
    else buf.upload(v);
  };
  ++ds->ws_gen;
  ds->ws_jb = -1;   // invalid until every buffer and descriptor is in place
  ds->ws_ni = -1;
  ds->ws_prec = -1;
  ds->ws_sym = -1;
  ds->H.free();
  ds->HT.free();
  ds->data.free();
  ds->KB.free();
  if (!from_ht) alloc(ds->H, size_t(sum_nb) * Q * jb * es);
  alloc(ds->data, size_t(2 * ds->nbox + extra) * Q * size_t(ncol) * es);
  ds->ws_pipe = pipe;
  alloc(ds->KB, size_t(sum_nb) * ni);
  if (sym) alloc(ds->HT, size_t(sum_nb) * Q * ni * es);
  const int64_t box_stride = int64_t(Q) * ncol;
  const char* Obase = prec == OCCK_PREC_FP64 ? reinterpret_cast<const char*>(ds->O.p)
                                             : reinterpret_cast<const char*>(ds->Of.p);
  std::vector<GemmDesc> dh, dom, dl, dht, dlt;
  std::vector<GemmTile> th, tom, tl2, tht, tlt, tltw, tl2w;
  int64_t pad48 = 0, pad144 = 0;   // leaf functions as padded by 48- and 144-wide tiles
  for (int b = 0; b < nl; ++b) {
    const int nb = int(t->leaf_funcs[b].size());
    pad48 += (nb + 47) / 48 * 48;
    pad144 += (nb + 143) / 144 * 144;
    const int64_t hoff = ds->f_off[b] * Q * jb;   // H^B[t][q][j], ld Q*jb (elements)
    const int32_t* g = ds->funcs.p + ds->f_off[b];
    const char* mloc = ds->data.p + int64_t(ds->nbox + ds->leaf_box[b]) * box_stride * es;
    for (int q = 0; q < Q; ++q) {  // H_q = O^B_q C_B[:, J]
      GemmDesc d{};
      d.A = Obase + (ds->O_off[b] + int64_t(q) * nb * nb) * es;
      d.sam = nb;
      d.sak = 1;
      d.gidx = g;
      d.C = from_ht ? nullptr : ds->H.p + (hoff + int64_t(q) * jb) * es;
      d.ldc = int64_t(Q) * jb;
      d.M = nb;
      d.N = jb;
      d.K = nb;
      if (!from_ht) {
        tiles_for<GemmRows48>(th, int(dh.size()), d.M, d.N);
        dh.push_back(d);
      }
      if (sym) {   // HT_q[i][t], column-major store
        GemmDesc e = d;
        e.C = ds->HT.p + (ds->f_off[b] * Q * ni + int64_t(q) * ni * nb) * es;
        e.ldc = 1;
        e.ldcn = nb;
        e.N = ni;
        tiles_for<GemmRows48>(tht, int(dht.size()), e.M, e.N);
        dht.push_back(e);
      }
    }
    if (from_ht) {  // Omega[(q,j), i] = sum_t HT_q[jstart + j][t] C[f(t), i0+i], one problem per q
      for (int q = 0; q < Q; ++q) {
        GemmDesc d{};
        d.A = ds->HT.p + (ds->f_off[b] * Q * ni + int64_t(q) * ni * nb) * es;
        d.sam = nb;
        d.sak = 1;
        d.gidx = g;
        d.C = ds->data.p + (int64_t(ds->leaf_box[b]) * box_stride + int64_t(q) * jb * ni) * es;
        d.ldc = ni;
        d.M = jb;
        d.N = ni;
        d.K = nb;
        tiles_for(tom, int(dom.size()), d.M, d.N);
        dom.push_back(d);
      }
    } else {  // Omega[(q,j), i] = sum_t H[t][(q,j)] C[f(t), i0+i]
      GemmDesc d{};
      d.A = ds->H.p + hoff * es;
      d.sam = 1;
      d.sak = int64_t(Q) * jb;
      d.gidx = g;
      d.C = ds->data.p + int64_t(ds->leaf_box[b]) * box_stride * es;
      d.ldc = ni;
      d.M = Q * jb;
      d.N = ni;
      d.K = nb;
      tiles_for(tom, int(dom.size()), d.M, d.N);
      dom.push_back(d);
    }
    if (from_ht) {  // KB[r, i] (+)= sum_q sum_j HT_q[jstart + j][r] Mloc[(q,j), i]: K segments q
      GemmDesc d{};
      d.A = ds->HT.p + ds->f_off[b] * Q * ni * es;
      d.sam = 1;
      d.sak = nb;
      d.sa_seg = int64_t(ni) * nb;
      d.B = mloc;
      d.ldb = ni;
      d.sb_seg = int64_t(jb) * ni;
      d.nseg = Q;
      d.C = ds->KB.p + ds->f_off[b] * ni;
      d.ldc = ni;
      d.M = nb;
      d.N = ni;
      d.K = jb;
      tiles_for<GemmRows48>(tl2, int(dl.size()), d.M, d.N);
      tiles_for<GemmRows144>(tl2w, int(dl.size()), d.M, d.N);
      dl.push_back(d);
    } else {  // KB[r, i] (+)= sum_(q,j) H[r][(q,j)] Mloc[(q,j), i]
      GemmDesc d{};
      d.A = ds->H.p + hoff * es;
      d.sam = int64_t(Q) * jb;
      d.sak = 1;
      d.B = mloc;
      d.ldb = ni;
      d.C = ds->KB.p + ds->f_off[b] * ni;
      d.ldc = ni;
      d.M = nb;
      d.N = ni;
      d.K = Q * jb;
      tiles_for<GemmRows48>(tl2, int(dl.size()), d.M, d.N);
      tiles_for<GemmRows144>(tl2w, int(dl.size()), d.M, d.N);
      dl.push_back(d);
    }
    if (sym) {  // KB[r, jstart + j] += sum_q sum_i Mloc[(q,j), i] HT_q[i][r]: rows j, columns r
      GemmDesc d{};
      d.A = mloc;
      d.sam = ni;
      d.sak = 1;
      d.sa_seg = ncol;
      d.B = ds->HT.p + ds->f_off[b] * Q * ni * es;
      d.ldb = nb;
      d.sb_seg = int64_t(ni) * nb;
      d.nseg = Q;
      d.C = ds->KB.p + ds->f_off[b] * ni;
      d.ldc = 1;
      d.ldcn = ni;
      d.M = jb;
      d.N = nb;
      d.K = ni;
      tiles_for<GemmCols48>(tlt, int(dlt.size()), d.M, d.N);
      tiles_for<GemmCols144>(tltw, int(dlt.size()), d.M, d.N);
      dlt.push_back(d);
    }
  }
  // omega: the column tiles of one row tile adjacent (they share its panel of
  // H), a box's gathered rows of C reused from L2 by all its row tiles;
  // l2p: the row tiles of one column tile adjacent (they share its panel of
  // Mloc), H of the box reused from L2 by all its column tiles
  ds->omega_nt_start = chunked_tile_lists(tom, [](const GemmTile& x) { return std::make_tuple(x.prob, x.mt, x.nt); });
  ds->l2p_nt_start = chunked_tile_lists(tl2, [](const GemmTile& x) { return std::make_tuple(x.prob, x.nt, x.mt); });
  // whole-leaf tiles (a leaf's n_B rows in one tile, each Mloc panel read
  // once) when they pad the leaves by at most a tenth more than 48-row tiles
  // (the persistent batch kernel uses the 48-row lists)
  const bool wide = 10 * pad144 <= 11 * pad48;
  ds->l2pw_nt_start.clear();
  ds->t_l2pw.free();
  if (wide) {
    ds->l2pw_nt_start = chunked_tile_lists(tl2w, [](const GemmTile& x) { return std::make_tuple(x.prob, x.nt, x.mt); });
    upload(ds->t_l2pw, tl2w);
  }
  // l2pt: the j tiles sharing one HT panel adjacent
  auto by_leaf = [](const GemmTile& x, const GemmTile& y) {
    return std::make_tuple(x.prob, x.nt, x.mt) < std::make_tuple(y.prob, y.nt, y.mt);
  };
  std::stable_sort(tlt.begin(), tlt.end(), by_leaf);
  std::stable_sort(tltw.begin(), tltw.end(), by_leaf);
  upload(ds->d_half, dh);
  upload(ds->t_half, th);
  upload(ds->d_omega, dom);
  upload(ds->t_omega, tom);
  upload(ds->d_l2p, dl);
  upload(ds->t_l2p, tl2);
  ds->n_half = int(th.size());
  ds->n_omega = ds->omega_nt_start.size() > 1 ? ds->omega_nt_start[1] : 0;   // list 0: every tile
  ds->n_l2p = ds->l2p_nt_start.size() > 1 ? ds->l2p_nt_start[1] : 0;
  ds->d_ht.free();
  ds->t_ht.free();
  ds->d_l2pt.free();
  ds->t_l2pt.free();
  ds->t_l2ptw.free();
  ds->n_ht = ds->n_l2pt = ds->n_l2ptw = 0;
  if (sym) {
    upload(ds->d_ht, dht);
    upload(ds->t_ht, tht);
    upload(ds->d_l2pt, dlt);
    upload(ds->t_l2pt, tlt);
    ds->n_ht = int(tht.size());
    ds->n_l2pt = int(tlt.size());
    if (wide) {   // a whole leaf per tile: each Mloc panel is read once
      upload(ds->t_l2ptw, tltw);
      ds->n_l2ptw = int(tltw.size());
    }
  }
  ds->ws_jb = jb;
  ds->ws_ni = ni;
  ds->ws_prec = prec;
  ds->ws_sym = sym_mode;
}

// ops_perm (may be null; not with src_rank): the operators in class order,
// for the MFMA translations of trees with structural zeros.
template <class T>
void launch_translate(const Tree* t, const Pass& ps, T* data, int64_t box_stride, const ColMap& cm, const T* ops,
                      hipStream_t st, const int8_t* src_rank, const T* ops_perm) {
  const int Q = t->Q, KS = ksteps_of(Q);
  if (cm.nvalid <= 0 || ps.ntgt == 0) return;
  if (Q <= 9 && !src_rank) {   // vector ALU, FP64 operators and accumulators in every mode
    const double* ops64 = t->dev->ops.p;
    constexpr int NC = 1;   // columns per thread
    const int64_t nblocks = ((cm.nvalid + 256 * NC - 1) / (256 * NC)) * ps.ntgt;
    const int64_t grid = ((nblocks + 7) / 8) * 8;
    if (grid > 0x7fffffff) throw std::invalid_argument("translation grid too large; lower jblock");
#define OCCK_TV(QQ, SY)                                                                                         \
  hipLaunchKernelGGL((translate_vec_kernel<T, QQ, NC, SY>), dim3(unsigned(grid)), dim3(256), 0, st, data,         \
                     box_stride, cm, KS, ps.tgt_box.p, ps.src_ptr.p, ps.src_box.p, ps.src_op.p, ops64, ps.ntgt,   \
                     nblocks)
#define OCCK_TVQ(QQ)                        \
  switch (t->dev->op_sym) {                 \
    case 1: OCCK_TV(QQ, 1); break;          \
    case 2: OCCK_TV(QQ, 2); break;          \
    default: OCCK_TV(QQ, 0); break;         \
  }
    switch (Q) {
      case 1: OCCK_TV(1, 0); break;
      case 4: OCCK_TVQ(4); break;
      case 9: OCCK_TVQ(9); break;
      default: throw std::invalid_argument("unsupported Q");
    }
#undef OCCK_TVQ
#undef OCCK_TV
    HIP_OK(hipGetLastError());
    return;
  }
  const int64_t nct = (cm.nvalid + 255) / 256;
  const int64_t nblocks = nct * ps.ntgt;
  const int64_t grid = ((nblocks + 7) / 8) * 8;
  if (grid > 0x7fffffff) throw std::invalid_argument("translation grid too large; lower jblock");
  const bool permuted = ops_perm && !src_rank && t->dev->perm.p;
  const T* opsm = permuted ? ops_perm : ops;
  const int32_t* perm = permuted ? t->dev->perm.p : nullptr;
  const int8_t* pcls = permuted ? t->dev->pcls.p : nullptr;
#define OCCK_TR(MT)                                                                                            \
  if (permuted)                                                                                                \
    hipLaunchKernelGGL((translate_perm_kernel<T, MT>), dim3(unsigned(grid)), dim3(256), 0, st, data, box_stride, \
                       cm, Q, KS, ps.tgt_box.p, ps.src_ptr.p, ps.src_box.p, ps.src_op.p, opsm, ps.ntgt, nblocks, \
                       perm, pcls);                                                                            \
  else                                                                                                         \
    hipLaunchKernelGGL((translate_kernel<T, MT>), dim3(unsigned(grid)), dim3(256), 0, st, data, box_stride, cm, \
                       Q, KS, ps.tgt_box.p, ps.src_ptr.p, ps.src_box.p, ps.src_op.p, ops, ps.ntgt, nblocks, src_rank)
  switch (mtiles_of(Q)) {
    case 1: OCCK_TR(1); break;
    case 2: OCCK_TR(2); break;
    case 3: OCCK_TR(3); break;
    case 4: OCCK_TR(4); break;
    case 5: OCCK_TR(5); break;
    case 6: OCCK_TR(6); break;
    default: throw std::invalid_argument("unsupported Q");
  }
#undef OCCK_TR
  HIP_OK(hipGetLastError());
}

// the upward (up) or downward walk over every subtree below level lmin
// (setup built the programs)
// store_shift (downward): box rows added to every stored leaf; load_shift:
// box rows added to every leaf read (upward) or to every source read whose
// box lies in [src_lo, src_hi) (downward)
template <class T>
void launch_walk(const Tree* t, const int32_t* pptr, const WalkStep* prog, int nroots, int nlv, bool up, T* data,
                 int64_t box_stride, const ColMap& cm, const T* ops, hipStream_t st, int64_t store_shift = 0,
                 int64_t load_shift = 0, int32_t src_lo = 0, int32_t src_hi = 0) {
  if (cm.nvalid <= 0 || nroots == 0) return;
  const int Q = t->Q, KS = ksteps_of(Q);
  const int64_t nblocks = ((cm.nvalid + 255) / 256) * nroots;
  const int64_t grid = ((nblocks + 7) / 8) * 8;
  if (grid > 0x7fffffff) throw std::invalid_argument("translation grid too large; lower jblock");
  // chain-like trees: the x-axis structural zeros, or none
  const bool xaxis = t->dev->op_sym == 1;
#define OCCK_WS(QQ, NL, SY)                                                                                        \
  if (up)                                                                                                          \
    hipLaunchKernelGGL((up_walk_kernel<T, QQ, NL, SY>), dim3(unsigned(grid)), dim3(256), 0, st, data, box_stride,  \
                       cm, KS, pptr, prog, ops, nroots, nblocks, load_shift);                                      \
  else                                                                                                             \
    hipLaunchKernelGGL((down_walk_kernel<T, QQ, NL, SY>), dim3(unsigned(grid)), dim3(256), 0, st, data,            \
                       box_stride, cm, KS, pptr, prog, ops, nroots, nblocks, store_shift, load_shift, src_lo,  \
                       src_hi)
#define OCCK_W(QQ, NL)          \
  if (xaxis && QQ > 1) {        \
    OCCK_WS(QQ, NL, 1);         \
  } else {                      \
    OCCK_WS(QQ, NL, 0);         \
  }
#define OCCK_WQ(QQ)                                                        \
  switch (nlv) {                                                           \
    case 1: OCCK_W(QQ, 1); break;                                          \
    case 2: OCCK_W(QQ, 2); break;                                          \
    case 3: OCCK_W(QQ, 3); break;                                          \
    case 4: OCCK_W(QQ, 4); break;                                          \
    case 5: OCCK_W(QQ, 5); break;                                          \
    case 6: OCCK_W(QQ, 6); break;                                          \
    default: throw std::invalid_argument("tree walk: unsupported depth"); \
  }
  switch (Q) {
    case 1: OCCK_WQ(1); break;
    case 4: OCCK_WQ(4); break;
    case 9: OCCK_WQ(9); break;
    default: throw std::invalid_argument("tree walk: unsupported Q");
  }
#undef OCCK_WQ
#undef OCCK_W
#undef OCCK_WS
  HIP_OK(hipGetLastError());
}

// Whether tree_chain_kernel takes the translations of element type T: a
// chain (build_chain), every class's LDS image of the tree within the
// block's LDS, and the level above the leaves within the held items.
template <class T>
static bool tree_lds_fits(const Tree* t, const DeviceState* ds) {
  if (ds->chain_nlev == 0 || t->Q != 9 || ds->op_sym != 1 || ds->leaf_box.empty()) return false;
  if (ds->nbox > kTreeMaxBoxes) return false;
  // a downward level above the leaves: the boxes of one x parity over half the
  // threads, at most kTreeRounds items each
  const int C = tree_cols(int(sizeof(T)));
  return (ds->chain_nbelow + 1) / 2 * int64_t(C) <= int64_t(kTreeThreads / 2) * kTreeRounds;
}

// One launch per reflection class: leaf Omega rows (+ load_shift) in, leaf
// Mloc rows (+ store_shift) out.
template <class T>
static int launch_tree_lds(const Tree* t, DeviceState* ds, T* data, int64_t box_stride, const ColMap& cm,
                           hipStream_t st, int64_t load_shift, int64_t store_shift) {
  if (cm.nvalid <= 0) return 0;
  const int nl = t->nleaf();
  const int32_t leaf0 = ds->leaf_box[0];
#define OCCK_TREE(CL)                                                                                              \
  {                                                                                                                \
    constexpr int C = tree_cols(int(sizeof(T)));                                                                  \
    const int64_t ngroups = (cm.nvalid + C - 1) / C;                                                              \
    const int64_t grid = ((ngroups + 7) / 8) * 8;                                                                 \
    if (grid > 0x7fffffff) throw std::invalid_argument("translation grid too large; lower jblock");               \
    hipLaunchKernelGGL((tree_chain_kernel<T, CL>), dim3(unsigned(grid)), dim3(kTreeThreads), 0, st, data,        \
                       box_stride, cm, ds->chain.p, ds->chain_nlev, ds->ops_cls.p + ds->ops_cls_off[CL], leaf0,  \
                       nl, ds->nbox, load_shift, store_shift, ngroups);                                          \
  }
  OCCK_TREE(0);
  OCCK_TREE(1);
  OCCK_TREE(2);
  OCCK_TREE(3);
#undef OCCK_TREE
  HIP_OK(hipGetLastError());
  return 4;
}

template void launch_translate<double>(const Tree*, const Pass&, double*, int64_t, const ColMap&, const double*,
                                       hipStream_t, const int8_t*, const double*);
template void launch_translate<float>(const Tree*, const Pass&, float*, int64_t, const ColMap&, const float*,
                                      hipStream_t, const int8_t*, const float*);

void launch_to_float(const double* in, int64_t ldi, float* out, int64_t ldo, int64_t rows, int64_t cols,
                     hipStream_t st) {
  const int64_t n = rows * cols;
  const int64_t blocks = std::min<int64_t>((n + 255) / 256, 65536);
  if (n == 0) return;
  hipLaunchKernelGGL(to_float_kernel, dim3(unsigned(blocks)), dim3(256), 0, st, in, ldi, out, ldo, rows, cols);
  HIP_OK(hipGetLastError());
}

// FP32 copies of the per-tree operands for the mixed paths (made once).
void ensure_mixed_operands(Tree* t, hipStream_t st) {
  DeviceState* ds = t->dev;
  if (ds->Of.p) return;
  ds->Of.alloc(ds->O.n);
  ds->opsf.alloc(ds->ops.n);
  launch_to_float(ds->O.p, 0, ds->Of.p, 0, 1, int64_t(ds->O.n), st);
}

void device_free(Tree* t) {
  if (t->dev) free_state(t->dev);
  t->dev = nullptr;
}

static void free_state(DeviceState* ds) {
  for (hipEvent_t e : ds->ev_pool) (void)hipEventDestroy(e);
  ds->ev_pool.clear();
  for (hipEvent_t e : {ds->ev_mloc[0], ds->ev_mloc[1], ds->ev_l2p[0], ds->ev_l2p[1], ds->ev_omega[0],
                       ds->ev_omega[1], ds->ev_start, ds->ev_join})
    if (e) (void)hipEventDestroy(e);
  if (ds->st2) (void)hipStreamDestroy(ds->st2);
  ds->Of.free();
  ds->opsf.free();
  ds->Cf.free();
  ds->O.free();
  ds->funcs.free();
  ds->opparam.free();
  ds->ops.free();
  ds->perm.free();
  ds->pcls.free();
  ds->ops_perm.free();
  ds->opsf_perm.free();
  for (auto& p : ds->up) { p.tgt_box.free(); p.src_ptr.free(); p.src_box.free(); p.src_op.free(); }
  for (auto& p : ds->down) {
    p.tgt_box.free(); p.src_ptr.free(); p.src_box.free(); p.src_op.free(); p.rank.free(); p.ent_tgt.free();
    p.strength.free();
  }
  ds->box_norm.free();
  ds->rank_hist.free();
  ds->occ_ptr.free();
  ds->occ_row.free();
  ds->H.free();
  ds->HT.free();
  ds->data.free();
  ds->KB.free();
  ds->d_half.free(); ds->d_omega.free(); ds->d_l2p.free(); ds->d_ht.free(); ds->d_l2pt.free();
  ds->t_half.free(); ds->t_omega.free(); ds->t_l2p.free(); ds->t_ht.free(); ds->t_l2pt.free();
  ds->t_l2ptw.free();
  ds->t_l2pw.free();
  delete ds;
}

int auto_jblock(const Tree* t, int nj, int ni, size_t es, bool sym, int jmax) {
  const size_t cap = device_cap();
  const int Q = t->Q;
  int64_t sum_nb = 0;
  for (const auto& f : t->leaf_funcs) sum_nb += int64_t(f.size());
  int64_t nbox = 0;
  for (int lev = t->lmin; lev <= t->params.depth; ++lev) nbox += int64_t(t->boxes[lev].size());
  const size_t budget = std::min(cap / 2, size_t(32) << 30);
  int jb = std::min(nj, jmax);
  while (jb > 1) {
    if (workspace_need(sum_nb, Q, nbox, jb, ni, es, sym) <= budget) break;
    jb = (jb + 1) / 2;
  }
  return std::max(1, jb);
}

// Occupied-pair screening (localised orbitals).  With n_Ai the l1 norm of
// orbital i over the functions centred in leaf A (its home leaf) and
// W_AA' the largest Gaussian product factor exp(-ab/(a+b)|A-B|^2) of a
// screened function pair joining the two, the bound
//   b_ij = sum_(A,A') n_Aj W_AA' n_A'i >= sum_(t,u) K_tu |C_tj| |C_ui|
// holds over every screened pair (t, u); (i, j) is carried when b_ij >= tau.
// nrm[A][i] = n_Ai.
static __global__ void homenorm_kernel(const double* __restrict__ C, int64_t ldc, int i0, int ni,
                                       const int32_t* __restrict__ hfn, const int32_t* __restrict__ hoff,
                                       double* __restrict__ nrm) {
  const int a = blockIdx.y;
  const int i = int(blockIdx.x) * 256 + threadIdx.x;
  if (i >= ni) return;
  double s = 0.0;
  for (int e = hoff[a]; e < hoff[a + 1]; ++e) s += fabs(C[int64_t(hfn[e]) * ldc + i0 + i]);
  nrm[int64_t(a) * ni + i] = s;
}

// spread[A][i] = sum_A' W_AA' nrm[A'][i].
static __global__ void homespread_kernel(const double* __restrict__ nrm, int ni, const int32_t* __restrict__ wptr,
                                         const int32_t* __restrict__ widx, const double* __restrict__ wval,
                                         double* __restrict__ spread) {
  const int a = blockIdx.y;
  const int i = int(blockIdx.x) * 256 + threadIdx.x;
  if (i >= ni) return;
  double s = 0.0;
  for (int e = wptr[a]; e < wptr[a + 1]; ++e) s = fma(wval[e], nrm[int64_t(widx[e]) * ni + i], s);
  spread[int64_t(a) * ni + i] = s;
}

// last[j] = the largest i > j with b_ij = sum_A nrm[A][j] spread[A][i] >= thresh,
// j itself when none; one block per j.
static __global__ __launch_bounds__(256) void pairband_kernel(const double* __restrict__ nrm,
                                                              const double* __restrict__ spread, int nleaf, int ni,
                                                              double thresh, int32_t* __restrict__ last) {
  __shared__ double nj[1024];
  __shared__ int32_t best[256];
  const int j = blockIdx.x;
  const int nchunk = (nleaf + 1023) / 1024;
  int32_t mine = j;
  // i strides over the threads; each i sums every leaf chunk before its test
  if (nchunk == 1) {
    for (int a = threadIdx.x; a < nleaf; a += 256) nj[a] = nrm[int64_t(a) * ni + j];
    __syncthreads();
  }
  for (int ib = j + 1; ib < ni; ib += 256) {
    const int i = ib + int(threadIdx.x);
    double b = 0.0;
    for (int c = 0; c < nchunk; ++c) {
      const int a0 = c * 1024;
      const int na = min(1024, nleaf - a0);
      if (nchunk > 1) {
        __syncthreads();
        for (int a = threadIdx.x; a < na; a += 256) nj[a] = nrm[int64_t(a0 + a) * ni + j];
        __syncthreads();
      }
      if (i < ni)
        for (int a = 0; a < na; ++a) b = fma(nj[a], spread[int64_t(a0 + a) * ni + i], b);
    }
    if (i < ni && b >= thresh) mine = i;
  }
  best[threadIdx.x] = mine;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (int(threadIdx.x) < o) best[threadIdx.x] = max(best[threadIdx.x], best[threadIdx.x + o]);
    __syncthreads();
  }
  if (threadIdx.x == 0) last[j] = best[0];
}

static __global__ void zero_kernel(double* __restrict__ x, int64_t count) {
  for (int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; e < count; e += int64_t(gridDim.x) * blockDim.x)
    x[e] = 0.0;
}

// Host tables of the screening bound: the home leaf of every function (the
// leaf of its pair with itself, which sits on its centre) and the leaf-leaf
// factors W_AA'.
static void upload_home_tables(Tree* t, DeviceState* ds) {
  const int nl = t->nleaf();
  std::vector<int32_t> home(t->funcs.size(), -1);
  for (const Pair& p : t->pairs)
    if (p.r == p.s) home[size_t(p.r)] = p.leaf;
  std::vector<int32_t> hoff(size_t(nl) + 1, 0), hfn(t->funcs.size());
  for (size_t f = 0; f < home.size(); ++f) {
    if (home[f] < 0) throw std::runtime_error("pair screening: a function has no pair with itself");
    ++hoff[size_t(home[f]) + 1];
  }
  for (int a = 0; a < nl; ++a) hoff[size_t(a) + 1] += hoff[size_t(a)];
  std::vector<int32_t> fill(hoff.begin(), hoff.end() - 1);
  for (size_t f = 0; f < home.size(); ++f) hfn[size_t(fill[size_t(home[f])]++)] = int32_t(f);
  std::vector<std::unordered_map<int32_t, double>> w(static_cast<size_t>(nl));
  for (const Pair& p : t->pairs) {
    const Func& fr = t->funcs[size_t(p.r)];
    const Func& fs = t->funcs[size_t(p.s)];
    double d2 = 0.0;
    for (int d = 0; d < 3; ++d) d2 += (fr.c[d] - fs.c[d]) * (fr.c[d] - fs.c[d]);
    const double k = std::exp(-fr.exp * fs.exp / (fr.exp + fs.exp) * d2);
    double& e = w[size_t(home[size_t(p.r)])][home[size_t(p.s)]];
    e = std::max(e, k);
  }
  std::vector<int32_t> wptr(size_t(nl) + 1, 0), widx;
  std::vector<double> wval;
  for (int a = 0; a < nl; ++a) {
    std::vector<std::pair<int32_t, double>> row(w[size_t(a)].begin(), w[size_t(a)].end());
    std::sort(row.begin(), row.end());
    for (const auto& e : row) {
      widx.push_back(e.first);
      wval.push_back(e.second);
    }
    wptr[size_t(a) + 1] = int32_t(widx.size());
  }
  ds->home_off.upload(hoff);
  ds->home_fn.upload(hfn);
  ds->hw_ptr.upload(wptr);
  ds->hw_idx.upload(widx);
  ds->hw_val.upload(wval);
}

// The i end of every j batch under occupied-pair screening: the largest
// carried i of the batch's j (at least the batch's own end).  Copies ni
// integers to the host (the call synchronises its stream here).
static std::vector<int> pair_bands(Tree* t, DeviceState* ds, const double* C, int64_t ldc, int i0, int ni, int jb,
                                   double thresh, hipStream_t st) {
  const int nl = t->nleaf();
  if (!ds->home_off.p) upload_home_tables(t, ds);
  ds->band_nrm.alloc(size_t(nl) * size_t(ni));
  ds->band_spread.alloc(size_t(nl) * size_t(ni));
  ds->band_last.alloc(size_t(ni));
  const dim3 grid(unsigned((ni + 255) / 256), unsigned(nl));
  hipLaunchKernelGGL(homenorm_kernel, grid, dim3(256), 0, st, C, ldc, i0, ni, ds->home_fn.p, ds->home_off.p,
                     ds->band_nrm.p);
  hipLaunchKernelGGL(homespread_kernel, grid, dim3(256), 0, st, ds->band_nrm.p, ni, ds->hw_ptr.p, ds->hw_idx.p,
                     ds->hw_val.p, ds->band_spread.p);
  hipLaunchKernelGGL(pairband_kernel, dim3(unsigned(ni)), dim3(256), 0, st, ds->band_nrm.p, ds->band_spread.p, nl, ni,
                     thresh, ds->band_last.p);
  HIP_OK(hipGetLastError());
  std::vector<int32_t> last(static_cast<size_t>(ni));
  HIP_OK(hipMemcpyAsync(last.data(), ds->band_last.p, size_t(ni) * 4, hipMemcpyDeviceToHost, st));
  HIP_OK(hipStreamSynchronize(st));
  std::vector<int> band;
  for (int j0b = 0; j0b < ni; j0b += jb) {
    const int j1b = std::min(ni, j0b + jb);
    int e = j1b;
    for (int j = j0b; j < j1b; ++j) e = std::max(e, int(last[size_t(j)]) + 1);
    band.push_back(std::min(e, ni));
  }
  return band;
}

// The j batches.  Per batch J = [jstart, jstart + jb): half transform,
// Omega, upward, downward, L2P.
//
// Symmetric schedule (sym: the i and j ranges coincide).  Omega^B_q and
// hence every translated Mloc^B_q are symmetric in (i, j) (the AO multipole
// O^{tu} is symmetric in t, u), so batch J carries only the columns (j, i)
// with i >= jstart.  K_ri then takes two contractions per batch: l2p over the
// carried columns, K[r, i] += sum_(q,j in J) H[r,(q,j)] Mloc[(q,j), i] for
// i >= jstart, and the mirrored l2pt, K[r, j] += sum_q sum_(i >= jstart+jb)
// H_q[r, i] Mloc[(q,j), i] for j in J, which supplies the pairs (i, j) whose
// i lies in an earlier batch.  The diagonal block (i, j both in J) is
// carried in full and counted once.  H of the batch is not formed again:
// HT, formed once per call for every column, holds it (rows jstart + j).
//
// Two streams (symmetric schedule with both walks, two_streams): the MFMA
// contractions (Omega, L2P) run on the library's stream st2 and the
// translations, bound by memory traffic, on the caller's stream, so that
// Omega of batch k+1 and the L2P of batch k overlap the translations of
// batch k+1.  Odd batches keep their leaf Omega and leaf Mloc in the extra
// box rows after the Mloc (nleaf rows each), so that two batches are in
// flight.  Order: st waits for Omega of batch k before its upward walk and
// for the L2P of batch k-2 before its downward walk writes that batch's
// leaf Mloc rows; st2 waits for the downward walk of batch k before its
// L2P (which also frees the leaf Omega rows of batch k for batch k+2's
// Omega, issued after it on st2); st waits for st2's last L2P before the
// reduction.
template <int MODE>
static void run_batches(Tree* t, DeviceState* ds, const typename ModeT<MODE>::T* Cg, int64_t ldcg, int i0, int i1,
                        int j0, int j1, int jb, int ni, bool prof, hipStream_t st, const void* sel,
                        bool stop_after_up = false, bool sym = false, const std::vector<int>* band = nullptr,
                        bool two_streams = false, bool lds_tree = false) {
  using T = typename ModeT<MODE>::T;
  const int Q = t->Q;
  const int64_t ncol = int64_t(jb) * ni;
  const int64_t box_stride = int64_t(Q) * ncol;
  T* data = reinterpret_cast<T*>(ds->data.p);
  const T* ops = MODE == kModeF64 ? reinterpret_cast<const T*>(ds->ops.p) : reinterpret_cast<const T*>(ds->opsf.p);
  // the MFMA translations of trees with structural zeros (fixed ranks) use the class-ordered operators
  const T* ops_perm = nullptr;
  if (ds->perm.p && !sel)
    ops_perm = MODE == kModeF64 ? reinterpret_cast<const T*>(ds->ops_perm.p)
                                : reinterpret_cast<const T*>(ds->opsf_perm.p);
  const int nj = j1 - j0;
  const int nblk = (nj + jb - 1) / jb;
  // the whole tree of each column group in LDS, in place of the walks and level passes
  const bool tree = lds_tree && !sel && !stop_after_up && tree_lds_fits<T>(t, ds);
  if (tree) {   // its class-compact operators, from this call's FP64 operators
    const int64_t n = int64_t(ds->ops_cls.n);
    hipLaunchKernelGGL(opclass_kernel, dim3(unsigned((n + 255) / 256)), dim3(256), 0, st, ds->ops.p,
                       int(t->ops.size()), 9, ds->op_sym, ds->ops_cls.p);
    HIP_OK(hipGetLastError());
  }
  const bool pipe = two_streams && sym && !sel && !stop_after_up && ds->ws_pipe && ds->dnw_nroots > 0 &&
                    ds->upw_nroots > 0 && nblk > 1;
  hipStream_t stg = st;   // the stream of Omega and the L2P
  if (pipe) {
    if (!ds->st2) {
      HIP_OK(hipStreamCreateWithFlags(&ds->st2, hipStreamNonBlocking));   // default priority
      for (hipEvent_t* e : {&ds->ev_mloc[0], &ds->ev_mloc[1], &ds->ev_l2p[0], &ds->ev_l2p[1], &ds->ev_omega[0],
                            &ds->ev_omega[1], &ds->ev_start, &ds->ev_join})
        HIP_OK(hipEventCreateWithFlags(e, hipEventDisableTiming));
    }
    stg = ds->st2;
  }
  // box rows of the second leaf Omega and leaf Mloc regions (odd batches)
  const int nl = t->nleaf();
  const int32_t leaf0 = ds->leaf_box.empty() ? 0 : ds->leaf_box[0];   // first leaf box slot
  const int64_t omega_shift = int64_t(2) * ds->nbox + nl - leaf0;     // leaf Omega rows -> the second region
  const int64_t mloc_shift = nl;                                      // leaf Mloc rows -> the second region

  struct Batch {
    int64_t jrel, jstart, istart, iend;
    int jbk, ct0;
    bool odd;
    ColMap cm;
  };
  auto batch = [&](int kb) {
    Batch b;
    b.jrel = int64_t(kb) * jb;                      // first j of the batch, relative to j0
    b.jstart = j0 + b.jrel;
    b.istart = sym ? b.jrel : 0;                    // first carried i (relative to i0)
    b.jbk = int(std::min<int64_t>(jb, nj - b.jrel));
    b.odd = pipe && (kb & 1);
    // occupied-pair screening: the batch carries i in [istart, iend) only
    b.iend = band ? int64_t((*band)[size_t(kb)]) : int64_t(ni);
    b.cm.ncol = ncol;
    b.cm.ni = ni;
    b.cm.istart = b.istart;
    b.cm.iend = band ? b.iend : 0;
    // the symmetric schedule carries the batch's own j only (the last batch
    // may be short: its Omega rows past jbk are not formed)
    b.cm.nvalid = int64_t(sym ? b.jbk : jb) * (b.iend - b.istart);
    b.ct0 = int(b.istart / 64);                     // first column tile touching i >= istart
    return b;
  };

  // half transform (all-column schedule only) and Omega, on stream s
  auto omega = [&](int kb, const Batch& b, hipStream_t s) {
    if (!sym) {   // the symmetric schedule reads the batch's H out of HT
      ProfScope ps(ds, prof, OCCK_K_HALF, s);
      GemmRun r{};
      r.boff = b.jstart;
      r.blim = j1;
      r.ntiles = ds->n_half;
      hipLaunchKernelGGL((half_kernel<MODE>), dim3(gemm_grid(r.ntiles)), dim3(256), 0, s, ds->d_half.p,
                         ds->t_half.p, Cg, ldcg, r);
    }
    ProfScope ps(ds, prof, OCCK_K_OMEGA, s);
    GemmRun r{};
    r.boff = i0;
    r.blim = i1;
    r.nhi = band ? int(b.iend) : 0;
    r.tile0 = ds->omega_nt_start[size_t(b.ct0 / 4)];
    r.ntiles = ds->omega_nt_start[size_t(b.ct0 / 4) + 1] - r.tile0;
    if (sym) {   // per (leaf, q): rows j of HT_q from the batch's first j
      r.amoff = int32_t(b.jrel);
      r.mlim = b.jbk;
      r.coff = b.odd ? omega_shift * box_stride : 0;   // the batch's leaf Omega rows
      hipLaunchKernelGGL((omega_ht_kernel<MODE>), dim3(gemm_grid(r.ntiles)), dim3(256), 0, s, ds->d_omega.p,
                         ds->t_omega.p, Cg, ldcg, r);
    } else {
      hipLaunchKernelGGL((omega_kernel<MODE>), dim3(gemm_grid(r.ntiles)), dim3(256), 0, s, ds->d_omega.p,
                         ds->t_omega.p, Cg, ldcg, r);
    }
    (void)kb;
  };

  // upward passes on stream s
  auto upward = [&](const Batch& b, hipStream_t s) {
    if (tree) return;   // part of the in-LDS tree kernel
    ProfScope ps(ds, prof, OCCK_K_UP, s, ds->upw_nroots > 0 ? 1 + ds->upw_lroot - t->lmin : int(ds->up.size()));
    // ds->up holds levels D-1 down to lmin; the walk covers those at or below its root level
    size_t k0 = 0;
    if (ds->upw_nroots > 0) {
      ProfScope ps_w(ds, prof, OCCK_K_UP_WALK, s);
      launch_walk<T>(t, ds->upw_ptr.p, ds->upw_prog.p, ds->upw_nroots, ds->upw_nlv, true, data, box_stride, b.cm,
                     ops, s, 0, b.odd ? omega_shift : 0, 0, 0);
      k0 = size_t(t->params.depth - ds->upw_lroot);
    }
    for (size_t k = k0; k < ds->up.size(); ++k)
      launch_translate<T>(t, ds->up[k], data, box_stride, b.cm, ops, s, nullptr, ops_perm);
  };

  // learned ranks and downward passes on stream s; wait_before_walk is
  // called just before the downward walk
  auto downward = [&](const Batch& b, hipStream_t s, auto&& wait_before_walk) {
    if (sel) {
      ProfScope ps(ds, prof, OCCK_K_SELECT, s, 1 + int(ds->down.size()));
      learned_ranks<T>(t, ds, sel, data, box_stride, b.cm, s);
    }
    if (tree) {
      wait_before_walk();
      ProfScope ps(ds, prof, OCCK_K_DOWN, s, 4);
      ProfScope ps_t(ds, prof, OCCK_K_TREE, s, 4);
      launch_tree_lds<T>(t, ds, data, box_stride, b.cm, s, b.odd ? omega_shift : 0, b.odd ? mloc_shift : 0);
      return;
    }
    // ds->down holds levels lmin..D; the walk covers those at or below its root level
    const bool walk = !sel && ds->dnw_nroots > 0;
    const size_t k1 = walk ? size_t(ds->dnw_lroot - t->lmin) : ds->down.size();
    ProfScope ps(ds, prof, OCCK_K_DOWN, s, int(k1) + (walk ? 1 : 0));
    for (size_t k = 0; k < k1; ++k)
      launch_translate<T>(t, ds->down[k], data, box_stride, b.cm, ops, s, sel ? ds->down[k].rank.p : nullptr,
                          ops_perm);
    if (walk) {
      wait_before_walk();
      ProfScope ps_w(ds, prof, OCCK_K_DOWN_WALK, s);
      launch_walk<T>(t, ds->dnw_ptr.p, ds->dnw_prog.p, ds->dnw_nroots, ds->dnw_nlv, false, data, box_stride, b.cm,
                     ops, s, b.odd ? mloc_shift : 0, b.odd ? omega_shift : 0, leaf0, leaf0 + nl);
    }
  };

  // direct and mirrored L2P on stream s
  auto l2p = [&](int kb, const Batch& b, hipStream_t s) {
    const int64_t mshift = b.odd ? mloc_shift * box_stride : 0;   // the batch's leaf Mloc rows
    ProfScope ps(ds, prof, OCCK_K_L2P, s, sym && b.jrel + jb < b.iend ? 2 : 1);
    GemmRun r{};
    r.accumulate = (kb > 0 || band) ? 1 : 0;   // with screening KB starts cleared
    r.nlo = int(b.istart);
    r.nhi = band ? int(b.iend) : 0;
    r.bptr = mshift;
    ProfScope ps_d(ds, prof, OCCK_K_L2P_DIRECT, s);
    if (sym) {   // K segments q, k = j over the batch's own j, A out of HT
      r.akoff = int32_t(b.jrel);
      r.klim = b.jbk;
    }
    if (!ds->l2pw_nt_start.empty()) {
      r.tile0 = ds->l2pw_nt_start[size_t(b.ct0 / 4)];
      r.ntiles = ds->l2pw_nt_start[size_t(b.ct0 / 4) + 1] - r.tile0;
      if (sym)
        hipLaunchKernelGGL((l2p_ht_wide_kernel<MODE>), dim3(gemm_grid(r.ntiles)), dim3(256), 0, s, ds->d_l2p.p,
                           ds->t_l2pw.p, Cg, ldcg, r);
      else
        hipLaunchKernelGGL((l2p_wide_kernel<MODE>), dim3(gemm_grid(r.ntiles)), dim3(256), 0, s, ds->d_l2p.p,
                           ds->t_l2pw.p, Cg, ldcg, r);
    } else {
      r.tile0 = ds->l2p_nt_start[size_t(b.ct0 / 4)];
      r.ntiles = ds->l2p_nt_start[size_t(b.ct0 / 4) + 1] - r.tile0;
      if (sym)
        hipLaunchKernelGGL((l2p_ht_kernel<MODE>), dim3(gemm_grid(r.ntiles)), dim3(256), 0, s, ds->d_l2p.p,
                           ds->t_l2p.p, Cg, ldcg, r);
      else
        hipLaunchKernelGGL((l2p_kernel<MODE>), dim3(gemm_grid(r.ntiles)), dim3(256), 0, s, ds->d_l2p.p,
                           ds->t_l2p.p, Cg, ldcg, r);
    }
    ps_d.close();
    if (sym && b.jrel + jb < b.iend) {
      ProfScope ps_m(ds, prof, OCCK_K_L2P_MIRROR, s);
      GemmRun m{};
      m.accumulate = 1;
      m.klim = band ? int(b.iend) : 0;
      m.koff = b.jrel + jb;
      m.aptr = mshift;
      m.coff = b.jrel;
      m.mlim = b.jbk;
      if (ds->n_l2ptw > 0) {
        m.ntiles = ds->n_l2ptw;
        hipLaunchKernelGGL((l2pt_wide_kernel<MODE>), dim3(gemm_grid(m.ntiles)), dim3(256), 0, s, ds->d_l2pt.p,
                           ds->t_l2ptw.p, Cg, ldcg, m);
      } else {
        m.ntiles = ds->n_l2pt;
        hipLaunchKernelGGL((l2pt_kernel<MODE>), dim3(gemm_grid(m.ntiles)), dim3(256), 0, s, ds->d_l2pt.p,
                           ds->t_l2pt.p, Cg, ldcg, m);
      }
    }
  };

  if (sym) {   // HT for every column, once per call
    ProfScope ps(ds, prof, OCCK_K_HALF, st);
    ProfScope ps_ht(ds, prof, OCCK_K_HT, st);
    GemmRun r{};
    r.boff = i0;
    r.blim = i1;
    r.ntiles = ds->n_ht;
    hipLaunchKernelGGL((half_kernel<MODE>), dim3(gemm_grid(r.ntiles)), dim3(256), 0, st, ds->d_ht.p,
                       ds->t_ht.p, Cg, ldcg, r);
  }
  if (!pipe) {
    for (int kb = 0; kb < nblk; ++kb) {
      const Batch b = batch(kb);
      omega(kb, b, st);
      upward(b, st);
      if (stop_after_up) return;
      downward(b, st, [] {});
      l2p(kb, b, st);
      HIP_OK(hipGetLastError());
    }
    return;
  }
  // two streams; every wait below is issued after the record it waits for
  HIP_OK(hipEventRecord(ds->ev_start, st));          // HT (and any earlier work on st) before Omega
  HIP_OK(hipStreamWaitEvent(stg, ds->ev_start, 0));
  omega(0, batch(0), stg);
  HIP_OK(hipEventRecord(ds->ev_omega[0], stg));
  for (int kb = 0; kb < nblk; ++kb) {
    const Batch b = batch(kb);
    const int p = kb & 1;
    HIP_OK(hipStreamWaitEvent(st, ds->ev_omega[p], 0));
    upward(b, st);
    downward(b, st, [&] {
      if (kb >= 2) HIP_OK(hipStreamWaitEvent(st, ds->ev_l2p[p], 0));   // batch kb-2 has read these Mloc rows
    });
    HIP_OK(hipEventRecord(ds->ev_mloc[p], st));
    if (kb + 1 < nblk) {   // its leaf Omega rows were last read by batch kb-1, whose L2P precedes on st2
      omega(kb + 1, batch(kb + 1), stg);
      HIP_OK(hipEventRecord(ds->ev_omega[p ^ 1], stg));
    }
    HIP_OK(hipStreamWaitEvent(stg, ds->ev_mloc[p], 0));
    l2p(kb, b, stg);
    HIP_OK(hipEventRecord(ds->ev_l2p[p], stg));
    HIP_OK(hipGetLastError());
  }
  HIP_OK(hipEventRecord(ds->ev_join, stg));   // the caller's stream resumes after the last L2P
  HIP_OK(hipStreamWaitEvent(st, ds->ev_join, 0));
}

// half transform, Omega and the upward passes of one FP64 j batch [j0, j1)
// (the batch must fit the workspace: setup_workspace(t, j1 - j0, i1 - i0, FP64))
void run_upward_fp64(Tree* t, DeviceState* ds, const double* C, int64_t ldc, int i0, int i1, int j0, int j1,
                     hipStream_t st) {
  hipLaunchKernelGGL(opgen_kernel, dim3(unsigned(t->ops.size())), dim3(64), 0, st, ds->opparam.p, ds->ops.p, t->L,
                     t->Q);
  if (ds->perm.p)
    hipLaunchKernelGGL(opgen_perm_kernel, dim3(unsigned(t->ops.size())), dim3(64), 0, st, ds->opparam.p,
                       ds->ops_perm.p, t->L, t->Q, ds->perm.p);
  HIP_OK(hipGetLastError());
  run_batches<kModeF64>(t, ds, C, ldc, i0, i1, j0, j1, j1 - j0, i1 - i0, false, st, nullptr, true);
}

int32_t far_K(Tree* t, const double* C, int64_t ldc, int32_t nocc, int32_t i0, int32_t i1, int32_t j0,
              int32_t j1, const occk_far_opts* opts, double* K, int64_t ldk, void* stream) {
  const void* sel = opts->rank_mode == OCCK_RANK_LEARNED ? static_cast<const void*>(opts->selector) : nullptr;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  const int ni = i1 - i0, nj = j1 - j0;
  const int nbasis = t->nbasis;
  const int prec = opts->precision;
  const bool mixed = prec != OCCK_PREC_FP64;
  try {
    if (t->lmin < 0 || nj == 0 || ni == 0) {   // no far field: nothing to upload
      if (!opts->accumulate && ni > 0)
        hipLaunchKernelGGL(zero_cols_kernel, dim3(unsigned((ni + 255) / 256), unsigned(nbasis)), dim3(256), 0, st,
                           K, ldk, i0, int64_t(ni));
      HIP_OK(hipGetLastError());
      return OCCK_OK;
    }
    const size_t es = mixed ? 4 : 8;
    const bool sym = i0 == j0 && i1 == j1;   // symmetric schedule when the i and j ranges coincide
    // Automatic j batches of at most 256, or 128 where the FP64 call runs the
    // two-stream schedule (symmetric, fixed rank, both walks): twice the
    // batches give the two streams more to overlap (alkane chain at L = 2:
    // 91.6 against 94.0 ms per call; FP32 is slower with 128 and split-BF16
    // the same, and one stream gains nothing).
    const bool pipe_fp64 = !mixed && sym && !sel && opts->one_stream == 0 && opts->pair_thresh <= 0.0 &&
                           opts->lds_tree != 1 && walk_tree(t);
    const int jb = opts->jblock > 0 ? std::min<int>(opts->jblock, nj)
                                    : auto_jblock(t, nj, ni, es, sym, pipe_fp64 ? 128 : 256);
    {
      // host-side check before any HIP call: leaf multipole blocks and the
      // workspace of this batch width must fit under the device-byte cap
      int64_t sum_nb = 0, sum_nb2 = 0, nbox = 0;
      for (const auto& f : t->leaf_funcs) {
        sum_nb += int64_t(f.size());
        sum_nb2 += int64_t(f.size()) * int64_t(f.size());
      }
      for (int lev = t->lmin; lev <= t->params.depth; ++lev) nbox += int64_t(t->boxes[lev].size());
      const size_t need = size_t(sum_nb2) * size_t(t->Q) * 8 +
                          workspace_need(sum_nb, t->Q, nbox, jb, ni, es, sym, sym ? 2 * t->nleaf() : 0);
      if (need > device_cap()) throw std::bad_alloc();
    }
    if (!t->dev) upload_tree(t);
    DeviceState* ds = t->dev;
    if (mixed) ensure_mixed_operands(t, st);
    setup_workspace(t, jb, ni, prec, sym ? kWsSymHT : kWsPlain);
    const int Q = t->Q;
    const bool prof = t->profile != 0;
    {
      ProfScope ps(ds, prof, OCCK_K_OPGEN, st);
      hipLaunchKernelGGL(opgen_kernel, dim3(unsigned(t->ops.size())), dim3(64), 0, st, ds->opparam.p, ds->ops.p,
                         t->L, Q);
      if (ds->perm.p && !sel)   // the MFMA translations' operators in class order
        hipLaunchKernelGGL(opgen_perm_kernel, dim3(unsigned(t->ops.size())), dim3(64), 0, st, ds->opparam.p,
                           ds->ops_perm.p, t->L, Q, ds->perm.p);
      HIP_OK(hipGetLastError());
    }
    if (mixed) {
      ProfScope ps(ds, prof, OCCK_K_CONVERT, st, 2);
      launch_to_float(ds->ops.p, 0, ds->opsf.p, 0, 1, int64_t(ds->ops.n), st);
      if (ds->perm.p && !sel) {
        ds->opsf_perm.alloc(ds->ops_perm.n);
        launch_to_float(ds->ops_perm.p, 0, ds->opsf_perm.p, 0, 1, int64_t(ds->ops_perm.n), st);
      }
      ds->Cf.alloc(size_t(nbasis) * nocc);
      launch_to_float(C, ldc, ds->Cf.p, nocc, nbasis, nocc, st);
    }
    const bool two = opts->one_stream == 0;   // the L2P may overlap the next batch on a second stream
    const bool lt = opts->lds_tree == 1;   // the in-LDS tree kernel on chains, when asked for
    std::vector<int> band;
    const std::vector<int>* bp = nullptr;
    if (opts->pair_thresh > 0.0) {   // occupied-pair screening (checked: symmetric ranges)
      band = pair_bands(t, ds, C, ldc, i0, ni, jb, opts->pair_thresh, st);
      bp = &band;
      hipLaunchKernelGGL(zero_kernel, dim3(2048), dim3(256), 0, st, ds->KB.p, int64_t(ds->KB.n));
      ds->last_band_cols = 0;
      for (size_t k = 0; k < band.size(); ++k) {
        const int64_t jlo = int64_t(k) * jb;
        ds->last_band_cols += (std::min(int64_t(ni), jlo + jb) - jlo) * (band[k] - jlo);
      }
      ds->band_end.assign(band.begin(), band.end());
      ds->band_jb = jb;
    }
    if (prec == OCCK_PREC_FP64)
      run_batches<kModeF64>(t, ds, C, ldc, i0, i1, j0, j1, jb, ni, prof, st, sel, false, sym, bp, two, lt);
    else if (prec == OCCK_PREC_FP32)
      run_batches<kModeF32>(t, ds, ds->Cf.p, nocc, i0, i1, j0, j1, jb, ni, prof, st, sel, false, sym, bp, two, lt);
    else if (prec == OCCK_PREC_BF16X3)
      run_batches<kModeBF16x3>(t, ds, ds->Cf.p, nocc, i0, i1, j0, j1, jb, ni, prof, st, sel, false, sym, bp, two, lt);
    else
      run_batches<kModeBF16x6>(t, ds, ds->Cf.p, nocc, i0, i1, j0, j1, jb, ni, prof, st, sel, false, sym, bp, two, lt);
    {
      ProfScope ps(ds, prof, OCCK_K_REDUCE, st);
      hipLaunchKernelGGL(reduce_kernel, dim3(unsigned((ni + 255) / 256), unsigned(nbasis)), dim3(256), 0, st,
                         ds->KB.p, int64_t(ni), ds->occ_ptr.p, ds->occ_row.p, K, ldk, i0, opts->accumulate);
    }
    HIP_OK(hipGetLastError());
  } catch (const HipError& e) {
    set_error(e.what());
    return OCCK_EHIP;
  } catch (const std::bad_alloc&) {
    set_error("device workspace exceeds OCCK_MAX_DEVICE_BYTES or allocation failed");
    return OCCK_ENOMEM;
  }
  return OCCK_OK;
}

// --------------------------------------------------------------------------
// allocation-free variant of far_K
// --------------------------------------------------------------------------
// The workspace of an allocation-free call lives in this region.  Host code
// never uses the array's name as an address: the per-device address comes
// from hipGetSymbolAddress (scratch_base).
static __device__ __align__(256) unsigned char scratch[size_t(OCCK_NOALLOC_SCRATCH_BYTES)];

static std::mutex g_scratch_mu;
static void* g_scratch_ptr[64] = {};

// Device address of `scratch` on device dev (current), looked up once per device.
static char* scratch_base(int dev) {
  if (dev < 0 || dev >= 64) throw std::invalid_argument("device ordinal out of range for the scratch table");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    HIP_OK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) throw HipError("hipGetSymbolAddress returned a null scratch address");
    g_scratch_ptr[dev] = p;
  }
  return static_cast<char*>(g_scratch_ptr[dev]);
}

// The owned workspace of a DeviceState, moved aside while an allocation-free
// call places its own workspace in the scratch region, then moved back.
struct WorkspaceStash {
  int ws_jb = -1, ws_ni = -1, ws_prec = -1, ws_sym = -1;
  uint64_t ws_gen = 0;
  bool ws_pipe = false;
  DevBuf<char> H, data, HT;
  DevBuf<double> KB;
  DevBuf<GemmDesc> d_half, d_omega, d_l2p, d_ht, d_l2pt;
  DevBuf<GemmTile> t_half, t_omega, t_l2p, t_ht, t_l2pt, t_l2ptw, t_l2pw;
  int n_half = 0, n_omega = 0, n_l2p = 0, n_ht = 0, n_l2pt = 0, n_l2ptw = 0;
  std::vector<int32_t> l2pw_nt_start, omega_nt_start, l2p_nt_start;
};

static void swap_workspace(DeviceState* ds, WorkspaceStash& w) {
  using std::swap;
  swap(ds->ws_jb, w.ws_jb); swap(ds->ws_ni, w.ws_ni); swap(ds->ws_prec, w.ws_prec); swap(ds->ws_sym, w.ws_sym);
  swap(ds->ws_gen, w.ws_gen);
  swap(ds->ws_pipe, w.ws_pipe);
  swap(ds->H, w.H); swap(ds->data, w.data); swap(ds->HT, w.HT); swap(ds->KB, w.KB);
  swap(ds->d_half, w.d_half); swap(ds->d_omega, w.d_omega); swap(ds->d_l2p, w.d_l2p); swap(ds->d_ht, w.d_ht);
  swap(ds->d_l2pt, w.d_l2pt);
  swap(ds->t_half, w.t_half); swap(ds->t_omega, w.t_omega); swap(ds->t_l2p, w.t_l2p); swap(ds->t_ht, w.t_ht);
  swap(ds->t_l2pt, w.t_l2pt); swap(ds->t_l2ptw, w.t_l2ptw); swap(ds->t_l2pw, w.t_l2pw);
  swap(ds->n_half, w.n_half); swap(ds->n_omega, w.n_omega); swap(ds->n_l2p, w.n_l2p); swap(ds->n_ht, w.n_ht);
  swap(ds->n_l2pt, w.n_l2pt); swap(ds->n_l2ptw, w.n_l2ptw);
  swap(ds->l2pw_nt_start, w.l2pw_nt_start); swap(ds->omega_nt_start, w.omega_nt_start);
  swap(ds->l2p_nt_start, w.l2p_nt_start);
}

// FP64, fixed rank (checked by the caller).  Same steps and kernels as far_K;
// only the workspace placement differs.
int32_t far_K_noalloc(Tree* t, const double* C, int64_t ldc, int32_t nocc, int32_t i0, int32_t i1, int32_t j0,
                      int32_t j1, const occk_far_opts* opts, double* K, int64_t ldk, void* stream) {
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  const int ni = i1 - i0, nj = j1 - j0;
  const int nbasis = t->nbasis;
  try {
    if (t->lmin < 0 || nj == 0 || ni == 0) {   // no far field
      if (!opts->accumulate && ni > 0)
        hipLaunchKernelGGL(zero_cols_kernel, dim3(unsigned((ni + 255) / 256), unsigned(nbasis)), dim3(256), 0, st,
                           K, ldk, i0, int64_t(ni));
      HIP_OK(hipGetLastError());
      return OCCK_OK;
    }
    DeviceState* ds = t->dev;
    if (!ds) {
      set_error("occk_far_K_noalloc: the tree has no device copy yet; one occk_far_K call on the handle makes it");
      return OCCK_ESTATE;
    }
    int dev = -1;
    HIP_OK(hipGetDevice(&dev));
    if (dev != ds->device) {
      set_error("occk_far_K_noalloc: the tree's device copy is on another device");
      return OCCK_EINVAL;
    }
    char* base = scratch_base(dev);
    // earlier work on this stream may still read the region's tables
    HIP_OK(hipStreamSynchronize(st));
    const bool sym = i0 == j0 && i1 == j1;
    WorkspaceStash stash;
    swap_workspace(ds, stash);
    struct Restore {
      DeviceState* ds;
      WorkspaceStash& w;
      ~Restore() { swap_workspace(ds, w); }   // the views left in w are dropped, never freed
    } restore{ds, stash};
    int jb = opts->jblock > 0 ? std::min<int>(opts->jblock, nj) : std::min(nj, 256);
    for (;;) {
      ScratchArena arena{base, size_t(OCCK_NOALLOC_SCRATCH_BYTES), 0};
      try {
        setup_workspace(t, jb, ni, OCCK_PREC_FP64, sym ? kWsSymHT : kWsPlain, &arena);
        break;
      } catch (const ScratchFull& e) {
        if (opts->jblock > 0 || jb == 1) {
          set_error(std::string("occk_far_K_noalloc: ") + e.what() + " (j batch " + std::to_string(jb) + ")");
          return OCCK_ENOMEM;
        }
        jb = (jb + 1) / 2;
      }
    }
    hipLaunchKernelGGL(opgen_kernel, dim3(unsigned(t->ops.size())), dim3(64), 0, st, ds->opparam.p, ds->ops.p,
                       t->L, t->Q);
    if (ds->perm.p)
      hipLaunchKernelGGL(opgen_perm_kernel, dim3(unsigned(t->ops.size())), dim3(64), 0, st, ds->opparam.p,
                         ds->ops_perm.p, t->L, t->Q, ds->perm.p);
    HIP_OK(hipGetLastError());
    run_batches<kModeF64>(t, ds, C, ldc, i0, i1, j0, j1, jb, ni, false, st, nullptr, false, sym, nullptr, false,
                          opts->lds_tree == 1);
    hipLaunchKernelGGL(reduce_kernel, dim3(unsigned((ni + 255) / 256), unsigned(nbasis)), dim3(256), 0, st,
                       ds->KB.p, int64_t(ni), ds->occ_ptr.p, ds->occ_row.p, K, ldk, i0, opts->accumulate);
    HIP_OK(hipGetLastError());
  } catch (const HipError& e) {
    set_error(e.what());
    return OCCK_EHIP;
  }
  return OCCK_OK;
}

// --------------------------------------------------------------------------
// diagnostics
// --------------------------------------------------------------------------
// MFMA lane-layout probe: a one-hot A (1 at row ia, column ka) times a
// one-hot B (1 at row ka, column jb) gives D = e_ia e_jb^T; every lane stores
// its accumulator values.  kind 0: v_mfma_f64_16x16x4f64 (A[i][k] in lane
// i+16k), 1: v_mfma_f32_16x16x4f32 (same operand layout), 2:
// v_mfma_f32_16x16x32_bf16 (A[i][k] in lane i+16(k/8), element k%8; B[k][j]
// in lane j+16(k/8), element k%8).  out: [64 lanes][4].
__global__ void mfma_probe_kernel(double* out, int kind, int ia, int ka, int jb) {
  const int lane = threadIdx.x;
  if (kind == 0) {
    const double a = ((lane & 15) == ia && (lane >> 4) == ka) ? 1.0 : 0.0;
    const double b = ((lane & 15) == jb && (lane >> 4) == ka) ? 1.0 : 0.0;
    d4 acc = d4{0.0, 0.0, 0.0, 0.0};
    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
    for (int r = 0; r < 4; ++r) out[lane * 4 + r] = acc[r];
  } else if (kind == 1) {
    const float a = ((lane & 15) == ia && (lane >> 4) == ka) ? 1.0f : 0.0f;
    const float b = ((lane & 15) == jb && (lane >> 4) == ka) ? 1.0f : 0.0f;
    f4 acc = f4{0.f, 0.f, 0.f, 0.f};
    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc, 0, 0, 0);
    for (int r = 0; r < 4; ++r) out[lane * 4 + r] = acc[r];
  } else {
    bf16x8 a, b;
    for (int e = 0; e < 8; ++e) {
      const int k = 8 * (lane >> 4) + e;
      a[e] = ((lane & 15) == ia && k == ka) ? (__bf16)1.0f : (__bf16)0.0f;
      b[e] = ((lane & 15) == jb && k == ka) ? (__bf16)1.0f : (__bf16)0.0f;
    }
    f4 acc = f4{0.f, 0.f, 0.f, 0.f};
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc, 0, 0, 0);
    for (int r = 0; r < 4; ++r) out[lane * 4 + r] = acc[r];
  }
}

int32_t debug_mfma_probe(int kind, int ia, int ka, int jb, double* host_out) {
  try {
    double* d = nullptr;
    HIP_OK(hipMalloc(&d, 256 * sizeof(double)));
    hipLaunchKernelGGL(mfma_probe_kernel, dim3(1), dim3(64), 0, 0, d, kind, ia, ka, jb);
    HIP_OK(hipGetLastError());
    HIP_OK(hipMemcpy(host_out, d, 256 * sizeof(double), hipMemcpyDeviceToHost));
    HIP_OK(hipFree(d));
  } catch (const HipError& e) {
    set_error(e.what());
    return OCCK_EHIP;
  }
  return OCCK_OK;
}

// Copies one workspace buffer of the last call to host memory (synchronous).
// which: 0 ops, 1 H, 2 box data (Omega then Mloc), 3 KB.  *count receives the
// element count; host may be NULL to query it.
int32_t debug_buffer(Tree* t, int which, double* host, int64_t* count) {
  DeviceState* ds = t->dev;
  if (!ds) {
    set_error("no device state");
    return OCCK_ESTATE;
  }
  // element counts in doubles (FP64 path) or in the buffer's own element size
  const void* p = nullptr;
  size_t bytes = 0, es = 8;
  if (which == 0) { p = ds->ops.p; bytes = ds->ops.n * 8; }
  else if (which == 1) { p = ds->H.p; bytes = ds->H.n; es = ds->ws_prec == OCCK_PREC_FP64 ? 8 : 4; }
  else if (which == 2) { p = ds->data.p; bytes = ds->data.n; es = ds->ws_prec == OCCK_PREC_FP64 ? 8 : 4; }
  else { p = ds->KB.p; bytes = ds->KB.n * 8; }
  const size_t n = bytes / es;
  if (count) *count = int64_t(n);
  if (host && n) {
    try {
      HIP_OK(hipDeviceSynchronize());
      if (es == 8) {
        HIP_OK(hipMemcpy(host, p, bytes, hipMemcpyDeviceToHost));
      } else {
        std::vector<float> tmp(n);
        HIP_OK(hipMemcpy(tmp.data(), p, bytes, hipMemcpyDeviceToHost));
        for (size_t k = 0; k < n; ++k) host[k] = tmp[k];
      }
    } catch (const HipError& e) {
      set_error(e.what());
      return OCCK_EHIP;
    }
  }
  return OCCK_OK;
}

// Sums the recorded event pairs per kernel class (synchronises on them) and clears.
int32_t profile_read(Tree* t, double* ms, int64_t* launches) {
  for (int c = 0; c < OCCK_K_NCLASS; ++c) {
    if (ms) ms[c] = 0.0;
    if (launches) launches[c] = 0;
  }
  DeviceState* ds = t->dev;
  if (!ds) return OCCK_OK;
  try {
    for (size_t k = 0; k < ds->ev_class.size(); ++k) {
      const size_t i = ds->ev_idx[k];
      HIP_OK(hipEventSynchronize(ds->ev_pool[i + 1]));
      float e = 0.f;
      HIP_OK(hipEventElapsedTime(&e, ds->ev_pool[i], ds->ev_pool[i + 1]));
      if (ms) ms[ds->ev_class[k]] += double(e);
    }
    if (launches && !ds->launches.empty())
      for (int c = 0; c < OCCK_K_NCLASS; ++c) launches[c] = ds->launches[c];
  } catch (const HipError& e) {
    set_error(e.what());
    return OCCK_EHIP;
  }
  ds->ev_class.clear();
  ds->ev_idx.clear();
  ds->ev_used = 0;
  ds->launches.assign(OCCK_K_NCLASS, 0);
  return OCCK_OK;
}

int32_t pair_screen_info(Tree* t, int64_t* carried, int32_t* jblock, int32_t* band_end, int32_t cap, int32_t* nband) {
  const DeviceState* ds = t->dev;
  *carried = ds ? ds->last_band_cols : 0;
  *jblock = ds ? ds->band_jb : 0;
  *nband = ds ? int32_t(ds->band_end.size()) : 0;
  for (int32_t k = 0; k < std::min(cap, *nband); ++k) band_end[k] = ds->band_end[size_t(k)];
  return OCCK_OK;
}

int32_t workspace_info(Tree* t, int32_t* jblock, int64_t* bytes) {
  DeviceState* ds = t->dev;
  if (jblock) *jblock = ds ? ds->ws_jb : -1;
  if (bytes) {
    *bytes = 0;
    if (ds)
      *bytes = int64_t(ds->bytes + ds->H.n + ds->data.n + ds->KB.n * 8 + ds->ops.n * 8 + ds->opsf.n * 4 +
                       ds->Of.n * 4 + ds->Cf.n * 4);
  }
  return OCCK_OK;
}

}  // namespace occk
