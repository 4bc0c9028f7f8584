// Host-side setup of the far-field exchange (per geometry): screened AO pairs,
// the hierarchical box tree with neighbour and interaction lists (Theory
// section of Le & Shiozaki, arXiv:1708.05353), the translation-operator list,
// and the leaf AO multipole integrals of Eq. (8) in FP64 real form.
//
// AO multipoles: the product of two Gaussians is a Gaussian at
// P = (aA + bB)/(a+b); with u = r - P, the regular harmonic is re-centred by
// the addition theorem O_lm(u + P - X) = sum O_{l-l',m-m'}(P-X) O_{l'm'}(u),
// and for s/p functions only l' <= 2 survive the integration against the
// Gaussian, whose Cartesian moments are closed-form.
//
// Compile with -ffp-contract=off: pair centres and leaf indices must be the
// plain IEEE results of the documented formulas.
#include <algorithm>
#include <array>
#include <cmath>
#include <complex>
#include <map>
#include <stdexcept>

#include "occk_internal.hpp"

namespace occk {

using cplx = std::complex<double>;

void Tree::centre(int level, const std::array<int32_t, 3>& c, double out[3]) const {
  for (int d = 0; d < 3; ++d) {
    if ((params.split_mask >> d) & 1)
      out[d] = lo[d] + (double(c[d]) + 0.5) * h(level);
    else
      out[d] = mid[d];
  }
}

int32_t Tree::parent(int level, int32_t box) const {
  const auto& c = boxes[level][box];
  auto it = index[level - 1].find(coord_key(c[0] >> 1, c[1] >> 1, c[2] >> 1));
  return it->second;
}

// O_{l,m}(v) for 0 <= m <= l <= L (complex, Eq. 4a with the Condon-Shortley
// phase), by the recurrences
//   O_{l,l} = -(x - i y)/(2l) O_{l-1,l-1},  O_{l+1,l} = z O_{l,l},
//   O_{l+1,m} = ((2l+1) z O_{l,m} - r^2 O_{l-1,m}) / ((l+1)^2 - m^2).
static void regular_cplx(int L, const double v[3], cplx* out /* [(L+1)*(L+2)/2] at l*(l+1)/2+m */) {
  const double x = v[0], y = v[1], z = v[2];
  const double r2 = x * x + y * y + z * z;
  auto at = [](int l, int m) { return l * (l + 1) / 2 + m; };
  out[0] = 1.0;
  for (int m = 0; m <= L; ++m) {
    if (m > 0) out[at(m, m)] = -cplx(x, -y) / double(2 * m) * out[at(m - 1, m - 1)];
    if (m + 1 <= L) out[at(m + 1, m)] = z * out[at(m, m)];
    for (int l = m + 1; l + 1 <= L; ++l)
      out[at(l + 1, m)] = (double(2 * l + 1) * z * out[at(l, m)] - r2 * out[at(l - 1, m)]) /
                          double((l + 1) * (l + 1) - m * m);
  }
}

// --------------------------------------------------------------------------
// intrinsic multipoles I_{l'm'} = N_r N_s K_ab int pre(u) O_{l'm'}(u) e^{-p u^2} d^3u
// for l' <= 2, m' >= 0, where pre(u) is the product of the p-function factors.
// --------------------------------------------------------------------------
struct Poly {            // coefficients c[a][b][c] of x^a y^b z^c, degree <= 4
  double c[5][5][5];
  Poly() { std::fill(&c[0][0][0], &c[0][0][0] + 125, 0.0); }
};

static Poly mul(const Poly& p, const Poly& q) {
  Poly o;
  for (int a = 0; a < 5; ++a)
    for (int b = 0; a + b < 5; ++b)
      for (int c = 0; a + b + c < 5; ++c) {
        if (p.c[a][b][c] == 0.0) continue;
        for (int a2 = 0; a + a2 < 5; ++a2)
          for (int b2 = 0; a + a2 + b + b2 < 5; ++b2)
            for (int c2 = 0; a + a2 + b + b2 + c + c2 < 5; ++c2)
              o.c[a + a2][b + b2][c + c2] += p.c[a][b][c] * q.c[a2][b2][c2];
      }
  return o;
}

static double gauss_moment(int n, double p) {   // int u^n e^{-p u^2} du
  if (n & 1) return 0.0;
  double v = std::sqrt(M_PI / p);
  for (int k = 1; k < n; k += 2) v *= double(k) / (2.0 * p);
  return v;
}

static double integrate(const Poly& f, double p) {
  double g[5];
  for (int n = 0; n < 5; ++n) g[n] = gauss_moment(n, p);
  double s = 0.0;
  for (int a = 0; a < 5; ++a)
    for (int b = 0; a + b < 5; ++b)
      for (int c = 0; a + b + c < 5; ++c)
        if (f.c[a][b][c] != 0.0) s += f.c[a][b][c] * g[a] * g[b] * g[c];
  return s;
}

// Real and imaginary polynomial parts of O_{l'm'}(u), l' <= 2, m' >= 0 (Eq. 4a).
static void harmonic_polys(Poly re[6], Poly im[6]) {
  // order: (0,0) (1,0) (1,1) (2,0) (2,1) (2,2)
  re[0].c[0][0][0] = 1.0;
  re[1].c[0][0][1] = 1.0;                                         // z
  re[2].c[1][0][0] = -0.5; im[2].c[0][1][0] = 0.5;                // -(x - i y)/2
  re[3].c[0][0][2] = 0.5; re[3].c[2][0][0] = -0.25; re[3].c[0][2][0] = -0.25;  // (2z^2-x^2-y^2)/4
  re[4].c[1][0][1] = -0.5; im[4].c[0][1][1] = 0.5;                // -z (x - i y)/2
  re[5].c[2][0][0] = 0.125; re[5].c[0][2][0] = -0.125; im[5].c[1][1][0] = -0.25;  // (x - i y)^2/8
}

static void pair_multipole(const Tree& t, const Pair& pr, const double X[3], double* out /* [Q] */) {
  struct Tables {
    Poly re[6], im[6];
    Tables() { harmonic_polys(re, im); }
  };
  static const Tables tab;   // initialised once (thread-safe static)
  const Poly* hre = tab.re;
  const Poly* him = tab.im;
  const Func& fa = t.funcs[pr.r];
  const Func& fb = t.funcs[pr.s];
  const double a = fa.exp, b = fb.exp, p = a + b;
  double d2 = 0.0;
  for (int d = 0; d < 3; ++d) d2 += (fa.c[d] - fb.c[d]) * (fa.c[d] - fb.c[d]);
  const double pref = fa.norm * fb.norm * std::exp(-a * b / p * d2);
  Poly pre;
  pre.c[0][0][0] = 1.0;
  for (int which = 0; which < 2; ++which) {
    const Func& f = which ? fb : fa;
    for (int d = 0; d < 3; ++d) {
      if (!f.pw[d]) continue;
      Poly lin;
      lin.c[0][0][0] = pr.P[d] - f.c[d];
      if (d == 0) lin.c[1][0][0] = 1.0;
      if (d == 1) lin.c[0][1][0] = 1.0;
      if (d == 2) lin.c[0][0][1] = 1.0;
      pre = mul(pre, lin);
    }
  }
  const int L = t.L;
  const int lint = std::min(L, 2);
  cplx I[3][3];  // I[l'][m'] for m' >= 0
  int k = 0;
  for (int lp = 0; lp <= 2; ++lp)
    for (int mp = 0; mp <= lp; ++mp, ++k) {
      if (lp > lint) { I[lp][mp] = 0.0; continue; }
      I[lp][mp] = pref * cplx(integrate(mul(pre, hre[k]), p), integrate(mul(pre, him[k]), p));
    }
  auto Iget = [&](int lp, int mp) -> cplx {
    if (mp >= 0) return I[lp][mp];
    cplx v = std::conj(I[lp][-mp]);
    return (mp & 1) ? -v : v;
  };
  double dv[3] = {pr.P[0] - X[0], pr.P[1] - X[1], pr.P[2] - X[2]};
  cplx Od[(kMaxLTree + 1) * (kMaxLTree + 2) / 2];
  regular_cplx(L, dv, Od);
  auto Oget = [&](int l, int m) -> cplx {
    if (m >= 0) return Od[l * (l + 1) / 2 + m];
    cplx v = std::conj(Od[l * (l + 1) / 2 - m]);
    return (m & 1) ? -v : v;
  };
  for (int l = 0; l <= L; ++l)
    for (int m = 0; m <= l; ++m) {
      cplx s = 0.0;
      for (int lp = 0; lp <= std::min(l, lint); ++lp)
        for (int mp = -lp; mp <= lp; ++mp)
          if (std::abs(m - mp) <= l - lp) s += Oget(l - lp, m - mp) * Iget(lp, mp);
      if (m == 0) {
        out[rq0(l)] = s.real();
      } else {
        out[rqre(l, m)] = s.real();
        out[rqim(l, m)] = s.imag();
      }
    }
}

void leaf_multipoles(const Tree& t, int leaf, double* out) {
  const auto& fl = t.leaf_funcs[leaf];
  const int nb = int(fl.size());
  const int Q = t.Q;
  std::fill(out, out + size_t(Q) * nb * nb, 0.0);
  double X[3];
  t.centre(t.params.depth, t.boxes[t.params.depth][leaf], X);
  std::vector<double> tmp(Q);
  for (int32_t pi : t.leaf_pairs[leaf]) {
    const Pair& pr = t.pairs[pi];
    pair_multipole(t, pr, X, tmp.data());
    const int a = int(std::lower_bound(fl.begin(), fl.end(), pr.r) - fl.begin());
    const int b = int(std::lower_bound(fl.begin(), fl.end(), pr.s) - fl.begin());
    for (int q = 0; q < Q; ++q) out[(size_t(q) * nb + a) * nb + b] += tmp[q];
  }
}

void leaf_pair_multipoles(const Tree& t, int leaf, double* out) {
  const int Q = t.Q;
  double X[3];
  t.centre(t.params.depth, t.boxes[t.params.depth][leaf], X);
  size_t k = 0;
  for (int32_t pi : t.leaf_pairs[leaf]) pair_multipole(t, t.pairs[pi], X, out + (k++) * size_t(Q));
}

// --------------------------------------------------------------------------
// tree construction
// --------------------------------------------------------------------------
static void fail(const std::string& m) { throw std::invalid_argument(m); }

// x >= 0 with erfc(x) = tau (0 < tau < 1/2), by Newton's method on erfc from
// x0 = sqrt(-ln tau); erfc is convex and decreasing there, so the iterates
// increase monotonically to the root.
static double erfc_inverse(double tau) {
  double x = std::sqrt(-std::log(tau)) - 1.0;
  if (x < 0.0) x = 0.0;
  for (int it = 0; it < 100; ++it) {
    const double f = std::erfc(x) - tau;
    const double df = -2.0 / std::sqrt(M_PI) * std::exp(-x * x);
    const double nx = x - f / df;
    if (std::fabs(nx - x) <= 1e-15 * std::max(1.0, nx)) return nx;
    x = nx;
  }
  return x;
}

// Interaction lists by the extents of the charge distributions (Theory
// section, the near/far paragraph): a pair distribution of exponent
// p = a + b has extent e = erfc^-1(tau)/sqrt(p); a box's extent is the largest
// |P - X_box| + e over the distributions whose centres it holds; two boxes of
// one level are far when |X_a - X_b| > (1 + ws)(e_a + e_b).  Near lists are
// formed top down from the root (near itself): a box's candidates are the
// children of its parent's near boxes, the far ones form its interaction
// list, the rest its near list.
static void extent_lists(Tree& t, const std::vector<std::array<int32_t, 3>>& pc) {
  const occk_tree_params& p = t.params;
  const int D = p.depth;
  const double einv = erfc_inverse(p.ext_tau);
  std::vector<std::vector<double>> ext(size_t(D + 1));
  std::vector<std::vector<std::array<double, 3>>> X(size_t(D + 1));
  for (int lev = 0; lev <= D; ++lev) {
    ext[size_t(lev)].assign(t.boxes[lev].size(), 0.0);
    X[size_t(lev)].resize(t.boxes[lev].size());
    for (size_t b = 0; b < t.boxes[lev].size(); ++b) t.centre(lev, t.boxes[lev][b], X[size_t(lev)][b].data());
  }
  for (size_t k = 0; k < t.pairs.size(); ++k) {
    const Pair& pr = t.pairs[k];
    const double e = einv / std::sqrt(t.funcs[size_t(pr.r)].exp + t.funcs[size_t(pr.s)].exp);
    for (int lev = 0; lev <= D; ++lev) {
      const int sh = D - lev;
      const int32_t b = t.index[lev].at(coord_key(pc[k][0] >> sh, pc[k][1] >> sh, pc[k][2] >> sh));
      const auto& x = X[size_t(lev)][size_t(b)];
      double d2 = 0.0;
      for (int d = 0; d < 3; ++d) d2 += (pr.P[d] - x[d]) * (pr.P[d] - x[d]);
      double& eb = ext[size_t(lev)][size_t(b)];
      eb = std::max(eb, std::sqrt(d2) + e);
    }
  }
  // children of every box, in box order
  std::vector<std::vector<std::vector<int32_t>>> kids(size_t(D + 1));
  for (int lev = 1; lev <= D; ++lev) {
    kids[size_t(lev - 1)].assign(t.boxes[lev - 1].size(), {});
    for (int32_t b = 0; b < int32_t(t.boxes[lev].size()); ++b) kids[size_t(lev - 1)][size_t(t.parent(lev, b))].push_back(b);
  }
  std::vector<std::vector<int32_t>> near_prev{{0}}, near_cur;
  t.il_ptr[0].assign(t.boxes[0].size() + 1, 0);
  for (int lev = 1; lev <= D; ++lev) {
    const auto& bx = t.boxes[lev];
    t.il_ptr[lev].assign(bx.size() + 1, 0);
    near_cur.assign(bx.size(), {});
    for (int32_t b = 0; b < int32_t(bx.size()); ++b) {
      const auto& xb = X[size_t(lev)][size_t(b)];
      const size_t e0 = t.il_idx[lev].size();
      for (int32_t q : near_prev[size_t(t.parent(lev, b))])
        for (int32_t b2 : kids[size_t(lev - 1)][size_t(q)]) {
          const auto& x2 = X[size_t(lev)][size_t(b2)];
          double d2 = 0.0;
          for (int d = 0; d < 3; ++d) d2 += (xb[d] - x2[d]) * (xb[d] - x2[d]);
          if (std::sqrt(d2) > (1.0 + p.ext_ws) * (ext[size_t(lev)][size_t(b)] + ext[size_t(lev)][size_t(b2)])) {
            for (int d = 0; d < 3; ++d)
              if (std::abs(bx[size_t(b)][d] - bx[size_t(b2)][d]) >= 64)
                fail("extent rule: an interaction-list displacement beyond 63 boxes");
            t.il_idx[lev].push_back(b2);
          } else {
            near_cur[size_t(b)].push_back(b2);
          }
        }
      std::sort(t.il_idx[lev].begin() + int64_t(e0), t.il_idx[lev].end());
      t.il_ptr[lev][size_t(b) + 1] = int32_t(t.il_idx[lev].size());
    }
    near_prev.swap(near_cur);
  }
  // near_prev holds the leaf level's near lists: the near field
  t.near_ptr.assign(1, 0);
  t.near_idx.clear();
  for (auto& v : near_prev) {
    std::sort(v.begin(), v.end());
    t.near_idx.insert(t.near_idx.end(), v.begin(), v.end());
    t.near_ptr.push_back(int32_t(t.near_idx.size()));
  }
}

Tree* build_tree(const occk_system* sys, const occk_tree_params* p) {
  if (!sys || !p) fail("null system or params");
  if (sys->natoms <= 0 || !sys->xyz) fail("natoms must be > 0 and xyz non-null");
  if (sys->nshell <= 0 || !sys->shell_atom || !sys->shell_l || !sys->shell_exp)
    fail("nshell must be > 0 and shell arrays non-null");
  if ((p->split_mask & 7) == 0 || (p->split_mask & ~7)) fail("split_mask must be a non-empty subset of {x,y,z}");
  if (p->depth < 1 || p->depth > 12) fail("depth must be in [1, 12]");
  if (p->ws < 0 || p->ws > 4) fail("ws must be in [0, 4]");
  if (p->lmax < 0 || p->lmax > kMaxLTree) fail("lmax must be in [0, 15]");
  if (std::isnan(p->pair_log_thresh) || p->pair_log_thresh <= 0) fail("pair_log_thresh must be > 0");
  if (p->near_rule != OCCK_NEAR_BOXES && p->near_rule != OCCK_NEAR_EXTENT) fail("near_rule must be 0 or 1");
  if (p->near_rule == OCCK_NEAR_EXTENT &&
      (!(p->ext_tau > 0.0) || !(p->ext_tau < 0.5) || !std::isfinite(p->ext_ws) || p->ext_ws <= -1.0 || p->ext_ws > 10.0))
    fail("extent rule: need 0 < ext_tau < 0.5 and -1 < ext_ws <= 10");
  for (int a = 0; a < 3 * sys->natoms; ++a)
    if (!std::isfinite(sys->xyz[a])) fail("non-finite coordinate");
  for (int s = 0; s < sys->nshell; ++s) {
    if (sys->shell_atom[s] < 0 || sys->shell_atom[s] >= sys->natoms) fail("shell_atom out of range");
    if (sys->shell_l[s] != 0 && sys->shell_l[s] != 1) fail("shell_l must be 0 or 1");
    if (!(sys->shell_exp[s] > 0) || !std::isfinite(sys->shell_exp[s])) fail("shell_exp must be finite and > 0");
  }

  Tree* tp = new Tree();
  Tree& t = *tp;
  try {
    t.params = *p;
    t.L = p->lmax;
    t.Q = (t.L + 1) * (t.L + 1);
    t.ndim = __builtin_popcount(unsigned(p->split_mask));
    // functions
    std::vector<int32_t> first(sys->nshell + 1, 0);
    for (int s = 0; s < sys->nshell; ++s) {
      first[s + 1] = first[s] + (sys->shell_l[s] == 0 ? 1 : 3);
      const double* A = sys->xyz + 3 * sys->shell_atom[s];
      const double e = sys->shell_exp[s];
      const int ncomp = sys->shell_l[s] == 0 ? 1 : 3;
      for (int k = 0; k < ncomp; ++k) {
        Func f{};
        for (int d = 0; d < 3; ++d) f.c[d] = A[d];
        f.exp = e;
        if (sys->shell_l[s] == 1) f.pw[k] = 1;
        f.norm = std::pow(2.0 * e / M_PI, 0.75) * (sys->shell_l[s] == 1 ? 2.0 * std::sqrt(e) : 1.0);
        f.shell = s;
        t.funcs.push_back(f);
      }
    }
    t.nbasis = int(t.funcs.size());
    t.shell_first.assign(first.begin(), first.end() - 1);
    t.shell_l.assign(sys->shell_l, sys->shell_l + sys->nshell);
    // screened ordered shell pairs -> function pairs
    const double thr = p->pair_log_thresh;
    const bool finite = std::isfinite(thr);
    for (int s1 = 0; s1 < sys->nshell; ++s1) {
      const double* A = sys->xyz + 3 * sys->shell_atom[s1];
      const double a = sys->shell_exp[s1];
      for (int s2 = 0; s2 < sys->nshell; ++s2) {
        const double* B = sys->xyz + 3 * sys->shell_atom[s2];
        const double b = sys->shell_exp[s2];
        double d2 = 0.0;
        for (int d = 0; d < 3; ++d) d2 += (A[d] - B[d]) * (A[d] - B[d]);
        const double val = (a * b / (a + b)) * d2;
        if (finite) {
          if (std::fabs(val - thr) <= 1e-9 * thr) fail("pair screening value within 1e-9 of the threshold");
          if (!(val <= thr)) continue;
        }
        for (int r = first[s1]; r < first[s1 + 1]; ++r)
          for (int s = first[s2]; s < first[s2 + 1]; ++s) {
            Pair pr{};
            pr.r = r;
            pr.s = s;
            for (int d = 0; d < 3; ++d) pr.P[d] = (a * A[d] + b * B[d]) / (a + b);
            t.pairs.push_back(pr);
          }
      }
    }
    if (t.pairs.empty()) fail("no AO pair survives screening");
    // root box
    double mn[3], mx[3];
    for (int d = 0; d < 3; ++d) { mn[d] = INFINITY; mx[d] = -INFINITY; }
    for (const Pair& pr : t.pairs)
      for (int d = 0; d < 3; ++d) { mn[d] = std::min(mn[d], pr.P[d]); mx[d] = std::max(mx[d], pr.P[d]); }
    double E = 0.0;
    for (int d = 0; d < 3; ++d)
      if ((p->split_mask >> d) & 1) E = std::max(E, mx[d] - mn[d]);
    const double delta = 0.05 * E + 1.0;
    for (int d = 0; d < 3; ++d) {
      t.mid[d] = 0.5 * (mn[d] + mx[d]);
      t.lo[d] = ((p->split_mask >> d) & 1) ? mn[d] - 0.35 * delta : 0.0;
    }
    t.W = E + delta;
    const int D = p->depth;
    const int32_t nside = int32_t(1) << D;
    const double hl = t.h(D);
    std::vector<std::array<int32_t, 3>> pc(t.pairs.size());
    for (size_t k = 0; k < t.pairs.size(); ++k) {
      std::array<int32_t, 3> c{0, 0, 0};
      for (int d = 0; d < 3; ++d) {
        if (!((p->split_mask >> d) & 1)) continue;
        const double u = (t.pairs[k].P[d] - t.lo[d]) / hl;
        const double f = std::floor(u);
        const double frac = u - f;
        if (std::min(frac, 1.0 - frac) < 1e-8) fail("a pair centre lies within 1e-8 h of a leaf boundary");
        int64_t iv = int64_t(f);
        iv = std::max<int64_t>(0, std::min<int64_t>(nside - 1, iv));
        c[d] = int32_t(iv);
      }
      pc[k] = c;
    }
    // levels
    t.boxes.assign(D + 1, {});
    t.index.assign(D + 1, {});
    for (int lev = 0; lev <= D; ++lev) {
      const int sh = D - lev;
      std::vector<std::array<int32_t, 3>> v;
      v.reserve(pc.size());
      for (const auto& c : pc) v.push_back({c[0] >> sh, c[1] >> sh, c[2] >> sh});
      std::sort(v.begin(), v.end());
      v.erase(std::unique(v.begin(), v.end()), v.end());
      t.boxes[lev] = v;
      for (int32_t b = 0; b < int32_t(v.size()); ++b) t.index[lev][coord_key(v[b][0], v[b][1], v[b][2])] = b;
    }
    for (size_t k = 0; k < t.pairs.size(); ++k)
      t.pairs[k].leaf = t.index[D].at(coord_key(pc[k][0], pc[k][1], pc[k][2]));
    t.il_ptr.assign(D + 1, {});
    t.il_idx.assign(D + 1, {});
    if (p->near_rule == OCCK_NEAR_EXTENT) {
      extent_lists(t, pc);
    } else {
    // interaction lists: non-near boxes whose parent is near the box's parent
    const int ws = p->ws;
    auto near = [ws](const std::array<int32_t, 3>& a, const std::array<int32_t, 3>& b) {
      int m = 0;
      for (int d = 0; d < 3; ++d) m = std::max(m, std::abs(a[d] - b[d]));
      return m <= ws;
    };
    for (int lev = 0; lev <= D; ++lev) {
      const auto& bx = t.boxes[lev];
      t.il_ptr[lev].assign(bx.size() + 1, 0);
      for (size_t b = 0; b < bx.size(); ++b) {
        if (lev > 0) {
          const std::array<int32_t, 3> pb{bx[b][0] >> 1, bx[b][1] >> 1, bx[b][2] >> 1};
          // candidates: children of the parent's near boxes
          for (int dz = -ws; dz <= ws; ++dz)
            for (int dy = -ws; dy <= ws; ++dy)
              for (int dx = -ws; dx <= ws; ++dx) {
                const int32_t q[3] = {pb[0] + dx, pb[1] + dy, pb[2] + dz};
                const int32_t pside = int32_t(1) << (lev - 1);
                bool bad = false;
                for (int d = 0; d < 3; ++d) {
                  if (!((p->split_mask >> d) & 1) && q[d] != 0) bad = true;
                  if (q[d] < 0 || q[d] >= pside) bad = true;
                }
                if (bad) continue;
                for (int oz = 0; oz < 2; ++oz)
                  for (int oy = 0; oy < 2; ++oy)
                    for (int ox = 0; ox < 2; ++ox) {
                      const int32_t cc[3] = {2 * q[0] + ox, 2 * q[1] + oy, 2 * q[2] + oz};
                      bool skip = false;
                      for (int d = 0; d < 3; ++d)
                        if (!((p->split_mask >> d) & 1) && cc[d] != 0) skip = true;
                      if (skip) continue;
                      auto it = t.index[lev].find(coord_key(cc[0], cc[1], cc[2]));
                      if (it == t.index[lev].end()) continue;
                      if (near(bx[b], t.boxes[lev][it->second])) continue;
                      t.il_idx[lev].push_back(it->second);
                    }
              }
          std::sort(t.il_idx[lev].begin() + t.il_ptr[lev][b], t.il_idx[lev].end());
        }
        t.il_ptr[lev][b + 1] = int32_t(t.il_idx[lev].size());
      }
    }
    }
    if (p->near_rule != OCCK_NEAR_EXTENT) {   // near field of the box-index rule: leaves within ws
      const int ws = p->ws;
      const auto& lv = t.boxes[D];
      t.near_ptr.assign(1, 0);
      t.near_idx.clear();
      for (size_t b = 0; b < lv.size(); ++b) {
        const size_t e0 = t.near_idx.size();
        for (int dz = -ws; dz <= ws; ++dz)
          for (int dy = -ws; dy <= ws; ++dy)
            for (int dx = -ws; dx <= ws; ++dx) {
              const int32_t c[3] = {lv[b][0] + dx, lv[b][1] + dy, lv[b][2] + dz};
              bool out = false;
              for (int d = 0; d < 3; ++d) {
                if (c[d] < 0 || c[d] >= nside) out = true;
                if (!((p->split_mask >> d) & 1) && c[d] != 0) out = true;
              }
              if (out) continue;
              auto it = t.index[D].find(coord_key(c[0], c[1], c[2]));
              if (it == t.index[D].end()) continue;
              t.near_idx.push_back(it->second);
            }
        std::sort(t.near_idx.begin() + int64_t(e0), t.near_idx.end());
        t.near_ptr.push_back(int32_t(t.near_idx.size()));
      }
    }
    for (int lev = 0; lev <= D; ++lev)
      if (t.lmin < 0 && !t.il_idx[lev].empty()) t.lmin = lev;
    // leaves
    const int nl = int(t.boxes[D].size());
    t.leaf_pairs.assign(nl, {});
    t.leaf_funcs.assign(nl, {});
    for (size_t k = 0; k < t.pairs.size(); ++k) t.leaf_pairs[t.pairs[k].leaf].push_back(int32_t(k));
    for (int b = 0; b < nl; ++b) {
      auto& f = t.leaf_funcs[b];
      for (int32_t k : t.leaf_pairs[b]) { f.push_back(t.pairs[k].r); f.push_back(t.pairs[k].s); }
      std::sort(f.begin(), f.end());
      f.erase(std::unique(f.begin(), f.end()), f.end());
    }
    // translation operators (levels lmin..D)
    if (t.lmin >= 0) {
      t.op_up.assign((D + 1) * 8, -1);
      t.op_down.assign((D + 1) * 8, -1);
      t.op_m2l.assign(D + 1, {});
      for (int lev = t.lmin + 1; lev <= D; ++lev) {
        const double hh = t.h(lev);
        for (int oct = 0; oct < 8; ++oct) {
          bool ok = true;
          OpDesc o{};
          for (int d = 0; d < 3; ++d) {
            const int bit = (oct >> d) & 1;
            if ((p->split_mask >> d) & 1)
              o.d[d] = (bit ? 0.5 : -0.5) * hh;
            else if (bit)
              ok = false;
            else
              o.d[d] = 0.0;
          }
          if (!ok) continue;
          o.type = kOpM2M;
          o.weighted = 0;
          t.op_up[lev * 8 + oct] = int32_t(t.ops.size());
          t.ops.push_back(o);
          o.type = kOpL2L;
          o.weighted = (lev == D);
          t.op_down[lev * 8 + oct] = int32_t(t.ops.size());
          t.ops.push_back(o);
        }
      }
      for (int lev = t.lmin; lev <= D; ++lev) {
        const double hh = t.h(lev);
        const auto& bx = t.boxes[lev];
        for (size_t b = 0; b < bx.size(); ++b)
          for (int32_t k = t.il_ptr[lev][b]; k < t.il_ptr[lev][b + 1]; ++k) {
            const auto& c2 = bx[t.il_idx[lev][k]];
            const int32_t dx = bx[b][0] - c2[0], dy = bx[b][1] - c2[1], dz = bx[b][2] - c2[2];
            const int64_t key = coord_key(dx + 64, dy + 64, dz + 64);
            if (t.op_m2l[lev].count(key)) continue;
            OpDesc o{};
            o.type = kOpM2L;
            o.weighted = (lev == D);
            o.d[0] = dx * hh;
            o.d[1] = dy * hh;
            o.d[2] = dz * hh;
            t.op_m2l[lev][key] = int32_t(t.ops.size());
            t.ops.push_back(o);
          }
      }
    }
    // structural nonzeros of the real-form M2M (= L2L) operator: output (l, m)
    // and input (l', mu), l' <= l, couple when |m -+ mu| <= l - l'
    int64_t nnz = 0;
    for (int l = 0; l <= t.L; ++l)
      for (int m = 0; m <= l; ++m)
        for (int lp = 0; lp <= l; ++lp)
          for (int mu = 0; mu <= lp; ++mu)
            if (std::abs(m - mu) <= l - lp || std::abs(m + mu) <= l - lp)
              nnz += int64_t(m == 0 ? 1 : 2) * (mu == 0 ? 1 : 2);
    t.m2m_nnz = nnz;
  } catch (...) {
    delete tp;
    throw;
  }
  return tp;
}

}  // namespace occk
