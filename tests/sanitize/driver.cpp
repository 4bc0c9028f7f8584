// Sanitized run of the host side of libocck: trees for a 1-D s-only chain, a
// 2-D s+p sheet and a 3-D cluster, every introspection call, the argument
// checks of occk_far_K and the handle checks.  Prints "sanitize driver OK"
// and exits 0 when every expectation holds.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "../../include/occk.h"

static int fails = 0;
#define EXPECT(c)                                                   \
  do {                                                              \
    if (!(c)) {                                                     \
      std::printf("FAILED %s:%d %s (%s)\n", __FILE__, __LINE__, #c, \
                  occk_last_error());                               \
      ++fails;                                                      \
    }                                                               \
  } while (0)

struct Sys {
  std::vector<double> xyz, ex;
  std::vector<int32_t> atom, l;
  occk_system view() const {
    return occk_system{int32_t(xyz.size() / 3), xyz.data(), int32_t(ex.size()), atom.data(), l.data(), ex.data()};
  }
  void add_atom(double x, double y, double z, const std::vector<double>& s_exp, const std::vector<double>& p_exp) {
    const int a = int(xyz.size() / 3);
    xyz.insert(xyz.end(), {x, y, z});
    for (double e : s_exp) { atom.push_back(a); l.push_back(0); ex.push_back(e); }
    for (double e : p_exp) { atom.push_back(a); l.push_back(1); ex.push_back(e); }
  }
};

static void exercise(const Sys& s, occk_tree_params p) {
  occk_system v = s.view();
  occk_tree* t = nullptr;
  EXPECT(occk_build_tree(&v, &p, &t) == OCCK_OK);
  if (!t) return;
  occk_tree_info_t inf;
  EXPECT(occk_tree_info(t, &inf) == OCCK_OK);
  occk_flops_t f;
  EXPECT(occk_tree_flops(t, 11, 7, 0, &f) == OCCK_OK);
  EXPECT(f.total == f.half + f.omega + f.m2m + f.m2l + f.l2l + f.l2p);
  EXPECT(occk_tree_flops(t, 11, 7, 1, &f) == OCCK_EINVAL);
  std::vector<int32_t> lc(size_t(inf.nleaf) * 3), lev(size_t(inf.n_il) + 1), tg(size_t(inf.n_il) + 1),
      sr(size_t(inf.n_il) + 1), pl(size_t(inf.npairs));
  EXPECT(occk_tree_export(t, lc.data(), lev.data(), tg.data(), sr.data(), pl.data()) == OCCK_OK);
  for (int32_t b = 0; b < inf.nleaf; ++b) {
    int32_t nb = 0;
    EXPECT(occk_tree_leaf(t, b, &nb, nullptr, nullptr) == OCCK_OK);
    std::vector<int32_t> fn(static_cast<size_t>(nb));
    std::vector<double> O(size_t(inf.ncomp) * size_t(nb) * size_t(nb));
    EXPECT(occk_tree_leaf(t, b, &nb, fn.data(), O.data()) == OCCK_OK);
    for (double x : O) EXPECT(std::isfinite(x));
  }
  EXPECT(occk_tree_leaf(t, inf.nleaf, nullptr, nullptr, nullptr) == OCCK_EINVAL);
  // occk_far_K argument checks (rejected before any device work)
  const double* C = reinterpret_cast<const double*>(0x100000);
  double* K = reinterpret_cast<double*>(0x90000000);
  const int n = 5;
  EXPECT(occk_far_K(t, nullptr, n, n, 0, n, 0, n, nullptr, K, n, nullptr) == OCCK_EINVAL);
  EXPECT(occk_far_K(t, C, n - 1, n, 0, n, 0, n, nullptr, K, n, nullptr) == OCCK_EINVAL);
  EXPECT(occk_far_K(t, C, n, n, 3, 2, 0, n, nullptr, K, n, nullptr) == OCCK_EINVAL);
  EXPECT(occk_far_K(t, C, n, n, 0, n, 0, n, nullptr, K, n - 1, nullptr) == OCCK_EINVAL);
  occk_far_opts bad{9, 0, nullptr, 0, 0};
  EXPECT(occk_far_K(t, C, n, n, 0, n, 0, n, &bad, K, n, nullptr) == OCCK_EINVAL);
  EXPECT(occk_free_tree(t) == OCCK_OK);
  EXPECT(occk_tree_info(t, &inf) == OCCK_EHANDLE);   // freed handle: rejected, not dereferenced
}

int main() {
  const double inf = INFINITY;
  {  // 1-D chain, 4 s shells per site, no screening
    Sys s;
    for (int k = 0; k < 20; ++k) s.add_atom(2.0 * k, 0, 0, {0.1, 0.4641588833612779, 2.154434690031884, 10.0}, {});
    exercise(s, occk_tree_params{1, 3, 2, 2, inf});
    exercise(s, occk_tree_params{1, 3, 1, 5, inf});
    exercise(s, occk_tree_params{1, 3, 0, 2, inf, OCCK_NEAR_EXTENT, 0.0, 1e-8});
  }
  {  // 2-D sheet with s and p shells, screened pairs
    Sys s;
    for (int a = 0; a < 6; ++a)
      for (int b = 0; b < 5; ++b)
        s.add_atom(2.4 * a + 1.2 * (b % 2), 2.1 * b, 0.0, {21.13, 1.774, 0.15}, {1.774, 0.15});
    exercise(s, occk_tree_params{3, 3, 1, 4, std::log(1e12)});
    exercise(s, occk_tree_params{3, 3, 0, 10, std::log(1e12), OCCK_NEAR_EXTENT, -0.1, 1e-8});
  }
  {  // 3-D cluster
    Sys s;
    unsigned seed = 12345u;
    auto rnd = [&seed]() { seed = seed * 1664525u + 1013904223u; return (seed >> 8) * (1.0 / 16777216.0); };
    for (int a = 0; a < 24; ++a) s.add_atom(12 * rnd(), 12 * rnd(), 12 * rnd(), {13.0, 0.12}, {1.249});
    exercise(s, occk_tree_params{7, 2, 1, 3, std::log(1e12)});
  }
  {  // rejected inputs
    Sys s;
    s.add_atom(0, 0, 0, {1.0}, {});
    s.add_atom(1, 0, 0, {-1.0}, {});
    occk_system v = s.view();
    occk_tree_params p{1, 2, 1, 2, inf};
    occk_tree* t = nullptr;
    EXPECT(occk_build_tree(&v, &p, &t) == OCCK_EINVAL && t == nullptr);
    p.lmax = 99;
    EXPECT(occk_build_tree(&v, &p, &t) == OCCK_EINVAL);
    EXPECT(occk_free_tree(nullptr) == OCCK_OK);
  }
  if (fails) return 1;
  std::printf("sanitize driver OK\n");
  return 0;
}
