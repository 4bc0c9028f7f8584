// Near-field occupied exchange with exact integrals (Le & Shiozaki,
// arXiv:1708.05353, Theory section: the pairs of charge distributions whose
// leaf boxes are near are not expanded in multipoles but computed exactly,
// alongside the far field), for uncontracted s and p Cartesian primitives on
// gfx950.
//
//   K^nf_ri = 2 sum_j sum_{(r,s) in B, (t,u) in B', B near B'} (rs|tu) C_sj C_tj C_ui
//           = sum_u X_ru C_ui,   X_ru = sum_{s,t} (rs|tu) D_st,   D = 2 C C^T
//
// Steps (all FP64, on the caller's stream):
//   transpose  CT = C^T
//   dense      D = C CT (FP64 MFMA grouped GEMM, one problem)
//   quartets   one wave per task: 64 bra shell pairs of one class (ss, sp,
//              ps, pp) in leaf B times a run of ket shell pairs of a near leaf
//              B' that share their second shell d; each lane forms the
//              integrals of its bra pair with every ket pair of the run by the
//              McMurchie-Davidson scheme (Hermite expansion coefficients E,
//              Hermite integrals R from the Boys function), contracts them
//              with D and keeps X[r, u] (r in its first shell, u in d) in
//              registers; the run's result goes to X with atomic adds
//   dense      K = X C (accumulate or overwrite)
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <map>
#include <new>
#include <stdexcept>
#include <vector>

#include "device.hpp"

namespace occk {

// One ordered pair of primitive shells (a on A, b on B) of a leaf.
struct SPair {
  double A[3], B[3], P[3];
  double p;       // a + b
  double pref;    // N_a N_b exp(-ab/p |A - B|^2)
  int32_t fa, fb; // first functions of the shells
  int32_t la, lb, sb, sd;   // angular momenta; shell ids of the second shell (ket runs)
};

// One wave task: bra pairs [bra0, bra0 + nbra) (one class), ket pairs
// [ket0, ket0 + nket) (one run: same second shell).
struct NTask {
  int32_t bra0, nbra, ket0, nket;
};

// ---------------------------------------------------------------------------
// Boys function F_n(T) = int_0^1 t^(2n) exp(-T t^2) dt, n = 0..N.
// T < kBoysTmax: F_N by its Taylor series about the nearest point T_g of a
// grid of step kBoysStep, F_N(T) = sum_k F_(N+k)(T_g) (T_g - T)^k / k!
// (dF_n/dT = -F_(n+1); |T_g - T| <= 0.05 and kBoysTerms terms leave a
// remainder below 1e-17 relative), from a table of F_m(T_g) formed once on
// the host; then the downward recurrence F_n = (2T F_(n+1) + e^-T)/(2n+1),
// which is stable.  T >= kBoysTmax: F_0 = (1/2) sqrt(pi/T) erf(sqrt(T)) and
// the upward recurrence F_(n+1) = ((2n+1) F_n - e^-T)/(2T), which loses
// nothing there.
constexpr int kBoysNmax = 4;                       // (pp|pp) needs F_0..F_4
constexpr int kBoysTerms = 9;                      // Taylor terms k = 0..8
constexpr int kBoysM = kBoysNmax + kBoysTerms;     // table columns m = 0..12
constexpr double kBoysTmax = 12.0, kBoysStep = 0.1;
constexpr int kBoysRows = 121;                     // T_g = 0, 0.1, ..., 12.0
__host__ __device__ constexpr double inv_int(int k) { return 1.0 / double(k); }

template <int N>
__device__ inline void boys(double T, double (&F)[N + 1], const double* __restrict__ tab) {
  static_assert(N <= kBoysNmax, "table columns");
  const double e = exp(-T);
  if (T < kBoysTmax) {
    const int g = int(T * (1.0 / kBoysStep) + 0.5);   // nearest grid point, 0..120
    const double d = double(g) * kBoysStep - T;       // T_g - T
    const double* row = tab + int64_t(g) * kBoysM + N;
    double s = row[kBoysTerms - 1];
#pragma unroll
    for (int k = kBoysTerms - 2; k >= 0; --k) s = fma(s, d * inv_int(k + 1), row[k]);
    F[N] = s;
#pragma unroll
    for (int n = N - 1; n >= 0; --n) F[n] = fma(2.0 * T, F[n + 1], e) * inv_int(2 * n + 1);
  } else {
    const double st = sqrt(T);
    F[0] = 0.886226925452758014 * erf(st) / st;   // sqrt(pi)/2
    const double h = 0.5 / T;
#pragma unroll
    for (int n = 0; n < N; ++n) F[n + 1] = (double(2 * n + 1) * F[n] - e) * h;
  }
}

// Host table of the Boys function for boys(): F_m(T_g), g < kBoysRows,
// m < kBoysM, by the series F_m(T) = e^-T sum_k (2T)^k / ((2m+1)(2m+3)...(2m+2k+1))
// in long double (all terms positive).
static std::vector<double> boys_table() {
  std::vector<double> tab(size_t(kBoysRows) * kBoysM);
  for (int g = 0; g < kBoysRows; ++g) {
    const long double T = (long double)g * (long double)kBoysStep;
    for (int m = 0; m < kBoysM; ++m) {
      long double term = 1.0L / (2 * m + 1), sum = term;
      for (int k = 1; k < 400 && term > 1e-24L * sum; ++k) {
        term *= 2.0L * T / (long double)(2 * m + 2 * k + 1);
        sum += term;
      }
      tab[size_t(g) * kBoysM + m] = double(expl(-T) * sum);
    }
  }
  return tab;
}

// Hermite coefficients of one Cartesian direction for powers i, j <= 1:
// E[i][j][t], t <= i + j, with the exponential factor taken out (E^00_0 = 1).
__device__ inline void hermite_e(double xpa, double xpb, double p, double (&E)[2][2][3]) {
  const double h = 0.5 / p;
  E[0][0][0] = 1.0; E[0][0][1] = 0.0; E[0][0][2] = 0.0;
  E[1][0][0] = xpa; E[1][0][1] = h;   E[1][0][2] = 0.0;
  E[0][1][0] = xpb; E[0][1][1] = h;   E[0][1][2] = 0.0;
  E[1][1][0] = xpa * xpb + h;
  E[1][1][1] = h * (xpa + xpb);
  E[1][1][2] = h * h;
}

// Hermite integrals R_{tuv} = R^0_{tuv}(alpha, R_PQ), t + u + v <= L.
template <int L>
struct RTable {
  double v[L + 1][L + 1][L + 1];
};

template <int L>
__device__ inline void hermite_r(double alpha, const double (&rpq)[3], RTable<L>& out, const double* __restrict__ btab) {
  double F[L + 1];
  boys<L>(alpha * (rpq[0] * rpq[0] + rpq[1] * rpq[1] + rpq[2] * rpq[2]), F, btab);
  // R^n_{tuv} for n from L down to 0; level n needs t + u + v <= L - n
  double Rn[L + 1][L + 1][L + 1][L + 1];
  double m2a = 1.0;
#pragma unroll
  for (int n = 0; n <= L; ++n) {
    Rn[n][0][0][0] = m2a * F[n];
    m2a *= -2.0 * alpha;
  }
#pragma unroll
  for (int n = L - 1; n >= 0; --n) {
#pragma unroll
    for (int t = 0; t <= L - n; ++t)
#pragma unroll
      for (int u = 0; u <= L - n - t; ++u)
#pragma unroll
        for (int w = 0; w <= L - n - t - u; ++w) {
          if (t + u + w == 0) continue;
          double r;
          if (t > 0) {
            r = rpq[0] * Rn[n + 1][t - 1][u][w];
            if (t > 1) r += double(t - 1) * Rn[n + 1][t - 2][u][w];
          } else if (u > 0) {
            r = rpq[1] * Rn[n + 1][t][u - 1][w];
            if (u > 1) r += double(u - 1) * Rn[n + 1][t][u - 2][w];
          } else {
            r = rpq[2] * Rn[n + 1][t][u][w - 1];
            if (w > 1) r += double(w - 1) * Rn[n + 1][t][u][w - 2];
          }
          Rn[n][t][u][w] = r;
        }
  }
#pragma unroll
  for (int t = 0; t <= L; ++t)
#pragma unroll
    for (int u = 0; u <= L - t; ++u)
#pragma unroll
      for (int w = 0; w <= L - t - u; ++w) out.v[t][u][w] = Rn[0][t][u][w];
}

// Cartesian powers of component k of a shell of momentum l (p: x, y, z).
__host__ __device__ constexpr int pw(int l, int k, int d) { return l == 0 ? 0 : (k == d ? 1 : 0); }

// X[r, u] += sum_{s, t} (rs|tu) D2[s][t] for one shell quartet, the bra's
// Hermite coefficients Eb (per direction) and the ket's Ek given.
template <int LA, int LB, int LC, int LD>
__device__ inline void quartet(const double (&Eb)[3][2][2][3], const double (&Ek)[3][2][2][3], const double (&rpq)[3],
                               double alpha, double scale, const double (&D2)[3][3], double (&X)[3][3],
                               const double* __restrict__ btab) {
  constexpr int L = LA + LB + LC + LD;
  RTable<L> R;
  hermite_r<L>(alpha, rpq, R, btab);
#pragma unroll
  for (int r = 0; r < 2 * LA + 1; ++r)
#pragma unroll
    for (int s = 0; s < 2 * LB + 1; ++s)
#pragma unroll
      for (int t = 0; t < 2 * LC + 1; ++t)
#pragma unroll
        for (int u = 0; u < 2 * LD + 1; ++u) {
          const int ix = pw(LA, r, 0), iy = pw(LA, r, 1), iz = pw(LA, r, 2);
          const int jx = pw(LB, s, 0), jy = pw(LB, s, 1), jz = pw(LB, s, 2);
          const int kx = pw(LC, t, 0), ky = pw(LC, t, 1), kz = pw(LC, t, 2);
          const int lx = pw(LD, u, 0), ly = pw(LD, u, 1), lz = pw(LD, u, 2);
          double acc = 0.0;
#pragma unroll
          for (int t1 = 0; t1 <= ix + jx; ++t1)
#pragma unroll
            for (int u1 = 0; u1 <= iy + jy; ++u1)
#pragma unroll
              for (int v1 = 0; v1 <= iz + jz; ++v1) {
                const double eb = Eb[0][ix][jx][t1] * Eb[1][iy][jy][u1] * Eb[2][iz][jz][v1];
                double inner = 0.0;
#pragma unroll
                for (int t2 = 0; t2 <= kx + lx; ++t2)
#pragma unroll
                  for (int u2 = 0; u2 <= ky + ly; ++u2)
#pragma unroll
                    for (int v2 = 0; v2 <= kz + lz; ++v2) {
                      const double ek = Ek[0][kx][lx][t2] * Ek[1][ky][ly][u2] * Ek[2][kz][lz][v2];
                      const double sg = ((t2 + u2 + v2) & 1) ? -1.0 : 1.0;
                      inner = fma(sg * ek, R.v[t1 + t2][u1 + u2][v1 + v2], inner);
                    }
                acc = fma(eb, inner, acc);
              }
          X[r][u] = fma(scale * acc, D2[s][t], X[r][u]);
        }
}

template <int LA, int LB, int LC, int LD>
__device__ inline void ket_step(const SPair& br, const double (&Eb)[3][2][2][3], const SPair& kt, const double* Dm,
                                int64_t n, double (&X)[3][3], const double* __restrict__ btab) {
  double Ek[3][2][2][3];
#pragma unroll
  for (int d = 0; d < 3; ++d) hermite_e(kt.P[d] - kt.A[d], kt.P[d] - kt.B[d], kt.p, Ek[d]);
  const double p = br.p, q = kt.p;
  const double alpha = p * q / (p + q);
  const double rpq[3] = {br.P[0] - kt.P[0], br.P[1] - kt.P[1], br.P[2] - kt.P[2]};
  // 2 pi^(5/2) / (p q sqrt(p + q)) times the prefactors, times 2 of D = 2 C C^T
  const double scale = 2.0 * 34.98683665524972497 / (p * q * sqrt(p + q)) * br.pref * kt.pref;
  double D2[3][3];
#pragma unroll
  for (int s = 0; s < 2 * LB + 1; ++s)
#pragma unroll
    for (int t = 0; t < 2 * LC + 1; ++t) D2[s][t] = Dm[int64_t(br.fb + s) * n + kt.fa + t];
  quartet<LA, LB, LC, LD>(Eb, Ek, rpq, alpha, scale, D2, X, btab);
}

// One wave per task.  Lane i takes bra pair bra0 + i (of class LA, LB); the
// ket run is uniform over the wave.  X is nbasis x nbasis, row-major.
template <int LA, int LB>
__global__ __launch_bounds__(64) void nf_quartet_kernel(const NTask* __restrict__ tasks,
                                                        const SPair* __restrict__ bra,
                                                        const SPair* __restrict__ ket,
                                                        const double* __restrict__ Dm, int64_t n,
                                                        double* __restrict__ Xm, const double* __restrict__ btab) {
  const NTask tk = tasks[blockIdx.x];
  const int lane = threadIdx.x;
  const bool ok = lane < tk.nbra;
  const SPair br = bra[tk.bra0 + (ok ? lane : 0)];
  double Eb[3][2][2][3];
#pragma unroll
  for (int d = 0; d < 3; ++d) hermite_e(br.P[d] - br.A[d], br.P[d] - br.B[d], br.p, Eb[d]);
  double X[3][3];
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int u = 0; u < 3; ++u) X[r][u] = 0.0;
  const int ld = ket[tk.ket0].lb;   // the run's second shell
  for (int e = 0; e < tk.nket; ++e) {
    const SPair kt = ket[tk.ket0 + e];
    const int lc = kt.la;
    if (ld == 0) {
      if (lc == 0) ket_step<LA, LB, 0, 0>(br, Eb, kt, Dm, n, X, btab);
      else ket_step<LA, LB, 1, 0>(br, Eb, kt, Dm, n, X, btab);
    } else {
      if (lc == 0) ket_step<LA, LB, 0, 1>(br, Eb, kt, Dm, n, X, btab);
      else ket_step<LA, LB, 1, 1>(br, Eb, kt, Dm, n, X, btab);
    }
  }
  if (!ok) return;
  const int fd = ket[tk.ket0].fb;
  for (int r = 0; r < 2 * LA + 1; ++r)
    for (int u = 0; u < 2 * ld + 1; ++u) atomicAdd(Xm + int64_t(br.fa + r) * n + fd + u, X[r][u]);
}

// out[j * ldo + r] = in[r * ldi + j] for r < rows, j < cols (32 x 32 tiles)
static __global__ void nf_transpose_kernel(const double* __restrict__ in, int64_t ldi, double* __restrict__ out,
                                           int64_t ldo, int64_t rows, int64_t cols) {
  __shared__ double tile[32][33];
  const int64_t r0 = int64_t(blockIdx.y) * 32, c0 = int64_t(blockIdx.x) * 32;
  for (int k = threadIdx.y; k < 32; k += blockDim.y) {
    const int64_t r = r0 + k, c = c0 + threadIdx.x;
    tile[k][threadIdx.x] = (r < rows && c < cols) ? in[r * ldi + c] : 0.0;
  }
  __syncthreads();
  for (int k = threadIdx.y; k < 32; k += blockDim.y) {
    const int64_t c = c0 + k, r = r0 + threadIdx.x;
    if (r < rows && c < cols) out[c * ldo + r] = tile[threadIdx.x][k];
  }
}

static __global__ void nf_zero_kernel(double* __restrict__ x, int64_t count) {
  for (int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; e < count; e += int64_t(gridDim.x) * blockDim.x)
    x[e] = 0.0;
}

// Plain FP64 GEMM C (+)= A B over a tile list (A k-contiguous, B row-major).
__global__ __launch_bounds__(256) void nf_dense_kernel(const GemmDesc* __restrict__ descs,
                                                       const GemmTile* __restrict__ tiles, GemmRun run) {
  gemm_grouped<kModeF64, true, false, double, GemmSquare, 2, 1>(descs, tiles, nullptr, 0, run);
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
struct NState {
  int device = -1;
  int64_t n = 0, nocc = 0;
  DevBuf<SPair> bra, ket;
  DevBuf<NTask> tasks[4];          // per bra class (la, lb) = (0,0), (0,1), (1,0), (1,1)
  int ntask[4] = {0, 0, 0, 0};
  DevBuf<double> D, X, CT;
  DevBuf<double> boys;             // Boys function table of boys()
  DevBuf<GemmDesc> gdesc;          // D = C CT, K = X C
  DevBuf<GemmTile> gtiles;
  int ntiles_d = 0, ntiles_k = 0;
  const double* c_ptr = nullptr;   // the C and K the descriptors point at
  int64_t ldc = 0;
  double* k_ptr = nullptr;
  int64_t ldk = 0;
  int64_t tasks_total = 0, quartets = 0;
};

void nstate_free(Tree* t) {
  delete t->ndev;
  t->ndev = nullptr;
}

static SPair make_spair(const Tree& t, int32_t sa, int32_t sb) {
  const Func& fa = t.funcs[size_t(t.shell_first[size_t(sa)])];
  const Func& fb = t.funcs[size_t(t.shell_first[size_t(sb)])];
  SPair q{};
  const double a = fa.exp, b = fb.exp, p = a + b;
  double ab2 = 0.0;
  for (int d = 0; d < 3; ++d) {
    q.A[d] = fa.c[d];
    q.B[d] = fb.c[d];
    q.P[d] = (a * fa.c[d] + b * fb.c[d]) / p;
    ab2 += (fa.c[d] - fb.c[d]) * (fa.c[d] - fb.c[d]);
  }
  q.p = p;
  q.pref = fa.norm * fb.norm * std::exp(-(a * b / p) * ab2);
  q.fa = t.shell_first[size_t(sa)];
  q.fb = t.shell_first[size_t(sb)];
  q.la = t.shell_l[size_t(sa)];
  q.lb = t.shell_l[size_t(sb)];
  q.sb = sb;
  q.sd = sb;
  return q;
}

static size_t nstate_need(const Tree* t, int64_t nocc) {
  const size_t n = size_t(t->nbasis);
  return (2 * n * n + n * size_t(nocc)) * 8 + t->pairs.size() * 2 * sizeof(SPair);
}

static void nstate_build(Tree* t, int64_t nocc) {
  if (nstate_need(t, nocc) > device_cap()) throw std::bad_alloc();
  NState* ns = new NState();
  try {
    HIP_OK(hipGetDevice(&ns->device));
    ns->n = t->nbasis;
    ns->nocc = nocc;
    const int nl = t->nleaf();
    // shell pairs of every leaf (all function pairs of a shell pair share its
    // centre and hence its leaf)
    std::vector<std::vector<std::pair<int32_t, int32_t>>> lsp(static_cast<size_t>(nl));
    for (int b = 0; b < nl; ++b) {
      std::vector<std::pair<int32_t, int32_t>> v;
      for (int32_t k : t->leaf_pairs[size_t(b)]) {
        const Pair& pr = t->pairs[size_t(k)];
        v.push_back({t->funcs[size_t(pr.r)].shell, t->funcs[size_t(pr.s)].shell});
      }
      std::sort(v.begin(), v.end());
      v.erase(std::unique(v.begin(), v.end()), v.end());
      lsp[size_t(b)] = v;
    }
    // bra order: per leaf, by class (la, lb); ket order: per leaf, by (second shell, la)
    std::vector<SPair> bra, ket;
    std::vector<std::array<int32_t, 5>> bra_off(static_cast<size_t>(nl));   // class c: [off[c], off[c+1])
    std::vector<std::vector<std::pair<int32_t, int32_t>>> runs(static_cast<size_t>(nl));   // (first, count) in ket
    for (int b = 0; b < nl; ++b) {
      for (int cls = 0; cls < 4; ++cls) {
        bra_off[size_t(b)][size_t(cls)] = int32_t(bra.size());
        for (const auto& sp : lsp[size_t(b)]) {
          const int c = 2 * t->shell_l[size_t(sp.first)] + t->shell_l[size_t(sp.second)];
          if (c == cls) bra.push_back(make_spair(*t, sp.first, sp.second));
        }
      }
      bra_off[size_t(b)][4] = int32_t(bra.size());
      std::vector<SPair> kv;
      for (const auto& sp : lsp[size_t(b)]) kv.push_back(make_spair(*t, sp.first, sp.second));
      std::stable_sort(kv.begin(), kv.end(), [](const SPair& x, const SPair& y) {
        return std::make_pair(x.sd, x.la) < std::make_pair(y.sd, y.la);
      });
      size_t e = 0;
      while (e < kv.size()) {
        size_t f = e;
        while (f < kv.size() && kv[f].sd == kv[e].sd) ++f;
        runs[size_t(b)].push_back({int32_t(ket.size() + e), int32_t(f - e)});
        e = f;
      }
      ket.insert(ket.end(), kv.begin(), kv.end());
    }
    ns->bra.upload(bra);
    ns->ket.upload(ket);
    ns->boys.upload(boys_table());
    // tasks: every near (leaf, leaf') pair, bra class, chunk of 64 bra pairs, ket run
    for (int cls = 0; cls < 4; ++cls) {
      std::vector<NTask> tl;
      for (int b = 0; b < nl; ++b) {
        const int32_t o0 = bra_off[size_t(b)][size_t(cls)], o1 = bra_off[size_t(b)][size_t(cls) + 1];
        for (int32_t e = t->near_ptr[size_t(b)]; e < t->near_ptr[size_t(b) + 1]; ++e) {
          const int32_t b2 = t->near_idx[size_t(e)];
          for (int32_t c0 = o0; c0 < o1; c0 += 64)
            for (const auto& rn : runs[size_t(b2)]) {
              tl.push_back({c0, std::min(64, o1 - c0), rn.first, rn.second});
              ns->quartets += int64_t(std::min(64, o1 - c0)) * rn.second;
            }
        }
      }
      ns->ntask[cls] = int(tl.size());
      ns->tasks_total += int64_t(tl.size());
      ns->tasks[cls].upload(tl);
    }
    const size_t n = size_t(ns->n);
    ns->D.alloc(n * n);
    ns->X.alloc(n * n);
    ns->CT.alloc(size_t(nocc) * n);
  } catch (...) {
    delete ns;
    throw;
  }
  t->ndev = ns;
}

static void tiles_square(std::vector<GemmTile>& tiles, int prob, int64_t M, int64_t N) {
  for (int mt = 0; mt < int((M + 63) / 64); ++mt)
    for (int nt = 0; nt < int((N + 63) / 64); ++nt) tiles.push_back({prob, mt, nt, 0});
}

// GEMM descriptors for D = C CT and K = X C with the caller's C and K
static void nstate_gemms(NState* ns, const double* C, int64_t ldc, double* K, int64_t ldk) {
  if (ns->c_ptr == C && ns->ldc == ldc && ns->k_ptr == K && ns->ldk == ldk && ns->gdesc.p) return;
  const int64_t n = ns->n, no = ns->nocc;
  std::vector<GemmDesc> d(2);
  d[0].A = C;             // D[r, s] = sum_j C[r, j] CT[j, s]
  d[0].sam = ldc;
  d[0].sak = 1;
  d[0].B = ns->CT.p;
  d[0].ldb = n;
  d[0].C = ns->D.p;
  d[0].ldc = n;
  d[0].M = int32_t(n);
  d[0].N = int32_t(n);
  d[0].K = int32_t(no);
  d[1].A = ns->X.p;       // K[r, i] = sum_u X[r, u] C[u, i]
  d[1].sam = n;
  d[1].sak = 1;
  d[1].B = C;
  d[1].ldb = ldc;
  d[1].C = K;
  d[1].ldc = ldk;
  d[1].M = int32_t(n);
  d[1].N = int32_t(no);
  d[1].K = int32_t(n);
  std::vector<GemmTile> tl;
  tiles_square(tl, 0, n, n);
  ns->ntiles_d = int(tl.size());
  tiles_square(tl, 1, n, no);
  ns->ntiles_k = int(tl.size()) - ns->ntiles_d;
  ns->gdesc.upload(d);
  ns->gtiles.upload(tl);
  ns->c_ptr = C;
  ns->ldc = ldc;
  ns->k_ptr = K;
  ns->ldk = ldk;
}

static inline unsigned grid8(int n) { return unsigned(((n + 7) / 8) * 8); }

int32_t near_K(Tree* t, const double* C, int64_t ldc, int32_t nocc, double* K, int64_t ldk, int32_t accumulate,
               void* stream) {
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  try {
    if (t->ndev && t->ndev->nocc != nocc) nstate_free(t);
    if (!t->ndev) nstate_build(t, nocc);
    NState* ns = t->ndev;
    nstate_gemms(ns, C, ldc, K, ldk);
    const int64_t n = ns->n;
    {
      dim3 grid(unsigned((nocc + 31) / 32), unsigned((n + 31) / 32));
      hipLaunchKernelGGL(nf_transpose_kernel, grid, dim3(32, 8), 0, st, C, ldc, ns->CT.p, n, n, int64_t(nocc));
    }
    GemmRun rd{};
    rd.ntiles = ns->ntiles_d;
    hipLaunchKernelGGL(nf_dense_kernel, dim3(grid8(rd.ntiles)), dim3(256), 0, st, ns->gdesc.p, ns->gtiles.p, rd);
    hipLaunchKernelGGL(nf_zero_kernel, dim3(4096), dim3(256), 0, st, ns->X.p, n * n);
    if (ns->ntask[0])
      hipLaunchKernelGGL((nf_quartet_kernel<0, 0>), dim3(unsigned(ns->ntask[0])), dim3(64), 0, st, ns->tasks[0].p,
                         ns->bra.p, ns->ket.p, ns->D.p, n, ns->X.p, ns->boys.p);
    if (ns->ntask[1])
      hipLaunchKernelGGL((nf_quartet_kernel<0, 1>), dim3(unsigned(ns->ntask[1])), dim3(64), 0, st, ns->tasks[1].p,
                         ns->bra.p, ns->ket.p, ns->D.p, n, ns->X.p, ns->boys.p);
    if (ns->ntask[2])
      hipLaunchKernelGGL((nf_quartet_kernel<1, 0>), dim3(unsigned(ns->ntask[2])), dim3(64), 0, st, ns->tasks[2].p,
                         ns->bra.p, ns->ket.p, ns->D.p, n, ns->X.p, ns->boys.p);
    if (ns->ntask[3])
      hipLaunchKernelGGL((nf_quartet_kernel<1, 1>), dim3(unsigned(ns->ntask[3])), dim3(64), 0, st, ns->tasks[3].p,
                         ns->bra.p, ns->ket.p, ns->D.p, n, ns->X.p, ns->boys.p);
    GemmRun rk{};
    rk.tile0 = ns->ntiles_d;
    rk.ntiles = ns->ntiles_k;
    rk.accumulate = accumulate;
    hipLaunchKernelGGL(nf_dense_kernel, dim3(grid8(rk.ntiles)), dim3(256), 0, st, ns->gdesc.p, ns->gtiles.p, rk);
    HIP_OK(hipGetLastError());
  } catch (const HipError& e) {
    set_error(e.what());
    return OCCK_EHIP;
  } catch (const std::bad_alloc&) {
    set_error("occk_near_K: device memory exceeds OCCK_MAX_DEVICE_BYTES or allocation failed");
    return OCCK_ENOMEM;
  }
  return OCCK_OK;
}

int32_t near_K_counts(Tree* t, int64_t* tasks, int64_t* quartets) {
  if (!t->ndev) return OCCK_ESTATE;
  if (tasks) *tasks = t->ndev->tasks_total;
  if (quartets) *quartets = t->ndev->quartets;
  return OCCK_OK;
}

}  // namespace occk
