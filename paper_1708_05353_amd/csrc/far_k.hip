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
#include <stdexcept>
#include <string>
#include <type_traits>
#include <vector>

#include "occk_internal.hpp"

typedef double d4 __attribute__((ext_vector_type(4)));

#define HIP_OK(x)                                                                    \
  do {                                                                               \
    hipError_t e_ = (x);                                                             \
    if (e_ != hipSuccess) throw HipError(std::string(#x) + ": " + hipGetErrorString(e_)); \
  } while (0)

namespace occk {

struct HipError : std::runtime_error {
  using std::runtime_error::runtime_error;
};

// --------------------------------------------------------------------------
// device-side descriptors
// --------------------------------------------------------------------------
struct GemmDesc {       // element types follow the kernel's mode (output: OutT)
  const void* A;       // A(m,k) = A[m*sam + k*sak]
  int64_t sam, sak;
  const void* B;       // B(k,n) = B[k*ldb + n]                (gidx == nullptr)
  int64_t ldb;
  const int32_t* gidx; // B(k,n) = Cuser[gidx[k]*ldcu + boff + n] (gather from C)
  void* C;             // C(m,n) = C[m*ldc + n]
  int64_t ldc;
  int32_t M, N, K, pad;
};
struct GemmTile {
  int32_t prob, mt, nt, pad;
};
struct OpParam {
  int32_t type, weighted;
  double d[3];
};

__host__ __device__ static inline int mtiles_of(int Q) { return (Q + 15) / 16; }
__host__ __device__ static inline int ksteps_of(int Q) { return (Q + 3) / 4; }
static inline int64_t opsize_of(int Q) { return int64_t(mtiles_of(Q)) * ksteps_of(Q) * 64; }

// --------------------------------------------------------------------------
// operator generation (FP64, one workgroup per operator)
// --------------------------------------------------------------------------
struct Cplx {
  double re, im;
};
__device__ inline Cplx cmul(Cplx a, Cplx b) { return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re}; }
__device__ inline Cplx cscale(Cplx a, double s) { return {a.re * s, a.im * s}; }

// table index for 0 <= m <= l
__device__ inline int tix(int l, int m) { return l * (l + 1) / 2 + m; }

// X_{l,m} for any sign of m from the m >= 0 table: X_{l,-m} = (-1)^m conj(X_{l,m})
__device__ inline Cplx tget(const Cplx* tab, int l, int m) {
  if (m >= 0) return tab[tix(l, m)];
  Cplx v = tab[tix(l, -m)];
  v.im = -v.im;
  if ((-m) & 1) { v.re = -v.re; v.im = -v.im; }
  return v;
}

// regular O_{l,m}(v), l <= L (Eq. 4a):
//   O_{m,m} = -(x - i y)/(2m) O_{m-1,m-1},  O_{m+1,m} = z O_{m,m},
//   O_{l+1,m} = ((2l+1) z O_{l,m} - r^2 O_{l-1,m}) / ((l+1)^2 - m^2)
__device__ void regular_table(int L, const double* v, Cplx* tab) {
  const double x = v[0], y = v[1], z = v[2], r2 = x * x + y * y + z * z;
  tab[0] = {1.0, 0.0};
  for (int m = 0; m <= L; ++m) {
    if (m > 0) tab[tix(m, m)] = cscale(cmul({x, -y}, tab[tix(m - 1, m - 1)]), -1.0 / (2.0 * m));
    if (m + 1 <= L) tab[tix(m + 1, m)] = cscale(tab[tix(m, m)], z);
    for (int l = m + 1; l + 1 <= L; ++l) {
      const double inv = 1.0 / double((l + 1) * (l + 1) - m * m);
      const Cplx a = tab[tix(l, m)], b = tab[tix(l - 1, m)];
      tab[tix(l + 1, m)] = {((2 * l + 1) * z * a.re - r2 * b.re) * inv, ((2 * l + 1) * z * a.im - r2 * b.im) * inv};
    }
  }
}

// irregular M_{l,m}(v), l <= L (Eq. 4b):
//   M_{0,0} = 1/r,  M_{m,m} = -(2m-1)(x + i y)/r^2 M_{m-1,m-1},
//   M_{m+1,m} = (2m+1) z M_{m,m}/r^2,
//   M_{l+1,m} = ((2l+1) z M_{l,m} - (l^2 - m^2) M_{l-1,m}) / r^2
__device__ void irregular_table(int L, const double* v, Cplx* tab) {
  const double x = v[0], y = v[1], z = v[2], r2 = x * x + y * y + z * z;
  const double ir2 = 1.0 / r2;
  tab[0] = {1.0 / sqrt(r2), 0.0};
  for (int m = 0; m <= L; ++m) {
    if (m > 0) tab[tix(m, m)] = cscale(cmul({x, y}, tab[tix(m - 1, m - 1)]), -(2.0 * m - 1.0) * ir2);
    if (m + 1 <= L) tab[tix(m + 1, m)] = cscale(tab[tix(m, m)], (2 * m + 1) * z * ir2);
    for (int l = m + 1; l + 1 <= L; ++l) {
      const Cplx a = tab[tix(l, m)], b = tab[tix(l - 1, m)];
      const double c = double(l * l - m * m);
      tab[tix(l + 1, m)] = {((2 * l + 1) * z * a.re - c * b.re) * ir2, ((2 * l + 1) * z * a.im - c * b.im) * ir2};
    }
  }
}

// complex coefficient c(l,m; l',m') of one translation
__device__ inline Cplx coef(int type, const Cplx* tab, int l, int m, int lp, int mp) {
  if (type == kOpM2M) {  // O_{l-l', m-m'}(d)
    if (lp > l || abs(m - mp) > l - lp) return {0.0, 0.0};
    return tget(tab, l - lp, m - mp);
  }
  if (type == kOpL2L) {  // O_{l'-l, m'-m}(d)
    if (lp < l || abs(mp - m) > lp - l) return {0.0, 0.0};
    return tget(tab, lp - l, mp - m);
  }
  Cplx v = tget(tab, l + lp, m + mp);  // (-1)^l M_{l+l', m+m'}(R)
  if (l & 1) { v.re = -v.re; v.im = -v.im; }
  return v;
}

// real component q -> (l, m, part): part 0 = (l,0) or Re, 1 = Im
__device__ inline void decode(int q, int& l, int& m, int& part) {
  l = 0;
  while ((l + 1) * (l + 1) <= q) ++l;
  const int k = q - l * l;
  if (k == 0) { m = 0; part = 0; }
  else { m = (k + 1) / 2; part = (k & 1) ? 0 : 1; }
}

// Real-form matrix entry T[row][col] of a translation acting on real-form
// vectors (m >= 0 components; negative m implied by X_{-m} = (-1)^m conj X_m).
__device__ double real_entry(int type, const Cplx* tab, int row, int col) {
  int l, m, pr, lp, mu, pc;
  decode(row, l, m, pr);
  decode(col, lp, mu, pc);
  const Cplx z1 = coef(type, tab, l, m, lp, mu);
  if (mu == 0) return pr == 0 ? z1.re : z1.im;
  Cplx z2 = coef(type, tab, l, m, lp, -mu);
  if (mu & 1) { z2.re = -z2.re; z2.im = -z2.im; }
  if (pc == 0) {  // coefficient of Re(x)
    const Cplx s{z1.re + z2.re, z1.im + z2.im};
    return pr == 0 ? s.re : s.im;
  }
  const Cplx d{z1.re - z2.re, z1.im - z2.im};  // coefficient of Im(x)
  return pr == 0 ? -d.im : d.re;
}

// L2P weights folded into leaf-level operators: K = 2 sum_lm O^{rj} Mloc^{ij}
// = sum_q w_q H_q Mloc_q with w = 2 for (l,0), 4 for Re, -4 for Im rows.
__device__ inline double l2p_weight(int q) {
  int l, m, p;
  decode(q, l, m, p);
  if (m == 0) return 2.0;
  return p == 0 ? 4.0 : -4.0;
}

// ops layout ("fragment order" of the FP64 MFMA A operand): element
// ((mt*KS + ks)*64 + lane) holds T[mt*16 + lane%16][ks*4 + lane/16].
__global__ __launch_bounds__(64) void opgen_kernel(const OpParam* __restrict__ params, double* __restrict__ ops,
                                                   int L, int Q) {
  __shared__ Cplx tab[(2 * kMaxL + 1) * (2 * kMaxL + 2) / 2];
  const OpParam p = params[blockIdx.x];
  if (threadIdx.x == 0) {
    if (p.type == kOpM2L) irregular_table(2 * L, p.d, tab);
    else regular_table(L, p.d, tab);
  }
  __syncthreads();
  const int MT = mtiles_of(Q), KS = ksteps_of(Q);
  double* out = ops + int64_t(blockIdx.x) * MT * KS * 64;
  for (int e = threadIdx.x; e < MT * KS * 64; e += 64) {
    const int lane = e & 63;
    const int frag = e >> 6;
    const int mt = frag / KS, ks = frag % KS;
    const int row = mt * 16 + (lane & 15), col = ks * 4 + (lane >> 4);
    double v = 0.0;
    if (row < Q && col < Q) {
      v = real_entry(p.type, tab, row, col);
      if (p.weighted) v *= l2p_weight(row);
    }
    out[e] = v;
  }
}

// --------------------------------------------------------------------------
// arithmetic modes of the contractions
//   kModeF64    FP64 operands, v_mfma_f64_16x16x4f64
//   kModeF32    FP32 operands, v_mfma_f32_16x16x4f32, FP32 accumulation
//   kModeBF16x3 FP32 operands split as x = hi + lo (bf16 each, round to
//               nearest even); a*b ~ hi_a hi_b + hi_a lo_b + lo_a hi_b on
//               v_mfma_f32_16x16x32_bf16 with FP32 accumulation
// MFMA layouts (checked with occk_debug_mfma_probe):
//   f64/f32 16x16x4: A[i][k] in lane i + 16k, B[k][j] in lane j + 16k;
//   bf16 16x16x32: A[i][k] in lane i + 16(k/8) element k%8, B likewise;
//   f64 D[i][j] in lane j + 16(i%4) element i/4 (rows interleaved),
//   f32 D[i][j] in lane j + 16(i/4) element i%4.
// --------------------------------------------------------------------------
//   kModeBF16x6 three-way split x = hi + mid + lo; six products
//               (hi hi, hi mid, mid hi, hi lo, lo hi, mid mid), ~2^-24 relative
enum { kModeF64 = 0, kModeF32 = 1, kModeBF16x3 = 2, kModeBF16x6 = 3 };
typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef short s8v __attribute__((ext_vector_type(8)));

template <int MODE> struct ModeT;
template <> struct ModeT<kModeF64> { using T = double; using Acc = d4; static constexpr int KT = 16; };
template <> struct ModeT<kModeF32> { using T = float; using Acc = f4; static constexpr int KT = 16; };
template <> struct ModeT<kModeBF16x3> { using T = float; using Acc = f4; static constexpr int KT = 32; };
template <> struct ModeT<kModeBF16x6> { using T = float; using Acc = f4; static constexpr int KT = 32; };

__device__ inline uint32_t bf16_rne_bits(float x) {   // bf16 bits (in the low half) of x, round to nearest even
  uint32_t u = __float_as_uint(x);
  u += 0x7fffu + ((u >> 16) & 1u);
  return u >> 16;
}

// x[e] -> hi[e] + lo[e] as bf16 vectors
__device__ inline void split8(const float* x, bf16x8& hi, bf16x8& lo) {
  s8v h, l;
  for (int e = 0; e < 8; ++e) {
    const uint32_t hb = bf16_rne_bits(x[e]);
    const float hf = __uint_as_float(hb << 16);
    h[e] = short(hb);
    l[e] = short(bf16_rne_bits(x[e] - hf));
  }
  hi = __builtin_bit_cast(bf16x8, h);
  lo = __builtin_bit_cast(bf16x8, l);
}

// x[e] -> hi[e] + mid[e] + lo[e] as bf16 vectors
__device__ inline void split8x3(const float* x, bf16x8& hi, bf16x8& mid, bf16x8& lo) {
  s8v h, m, l;
  for (int e = 0; e < 8; ++e) {
    const uint32_t hb = bf16_rne_bits(x[e]);
    const float r1 = x[e] - __uint_as_float(hb << 16);
    const uint32_t mb = bf16_rne_bits(r1);
    const float r2 = r1 - __uint_as_float(mb << 16);
    h[e] = short(hb);
    m[e] = short(mb);
    l[e] = short(bf16_rne_bits(r2));
  }
  hi = __builtin_bit_cast(bf16x8, h);
  mid = __builtin_bit_cast(bf16x8, m);
  lo = __builtin_bit_cast(bf16x8, l);
}

__device__ inline d4 mfma4(double a, double b, d4 c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }
__device__ inline f4 mfma4(float a, float b, f4 c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }

// output row of accumulator element r for lane group g = lane/16 inside a 16-row tile
template <class Acc> __device__ inline int acc_row(int g, int r);
template <> __device__ inline int acc_row<d4>(int g, int r) { return g + 4 * r; }
template <> __device__ inline int acc_row<f4>(int g, int r) { return 4 * g + r; }

// --------------------------------------------------------------------------
// grouped GEMM: C(m,n) (+)= sum_k A(m,k) B(k,n) over a list of problems;
// 64x64 output tile per 256-thread block, each wave a 32x32 quadrant (2x2
// MFMA tiles), K staged through LDS in steps of KT.
// --------------------------------------------------------------------------
template <int MODE, bool A_KCONTIG, class OutT>
__global__ __launch_bounds__(256) void gemm_kernel(const GemmDesc* __restrict__ descs,
                                                   const GemmTile* __restrict__ tiles,
                                                   const typename ModeT<MODE>::T* __restrict__ Cuser, int64_t ldcu,
                                                   int64_t boff, int64_t blim, int accumulate) {
  using T = typename ModeT<MODE>::T;
  using Acc = typename ModeT<MODE>::Acc;
  constexpr int KT = ModeT<MODE>::KT;
  constexpr int E = KT / 4;          // elements per thread per operand tile
  __shared__ T As[KT][64 + 1];
  __shared__ T Bs[KT][64 + 1];
  const GemmTile tl = tiles[blockIdx.x];
  const GemmDesc d = descs[tl.prob];
  const T* A = static_cast<const T*>(d.A);
  const int m0 = tl.mt * 64, n0 = tl.nt * 64;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = (wave & 1) * 32, wn = (wave >> 1) * 32;
  Acc acc[2][2];
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j) acc[i][j] = Acc{};
  // FP32 accumulators feeding an FP64 output are flushed into FP64 registers
  // every FLUSH K tiles, so FP32 rounding accumulates over at most FLUSH*KT terms.
  constexpr bool kFlush = std::is_same<OutT, double>::value && MODE != kModeF64;
  constexpr int FLUSH = 8;
  double acc64[kFlush ? 2 : 1][kFlush ? 2 : 1][kFlush ? 4 : 1];
  if constexpr (kFlush)
    for (int i = 0; i < 2; ++i)
      for (int j = 0; j < 2; ++j)
        for (int r = 0; r < 4; ++r) acc64[i][j][r] = 0.0;
  int ktile = 0;
  // A: k-contiguous -> row am = tid/4, k = (tid%4)*E ..; m-contiguous -> k = tid/(64/E), m = (tid%(64/E))*E ..
  // B: k = tid/(64/E), n = (tid%(64/E))*E ..
  constexpr int TPR = 64 / E;
  const int bk = tid / TPR, bn = (tid % TPR) * E;
  T ra[E], rb[E];
  auto load = [&](int k0) {
    if (A_KCONTIG) {
      const int am = tid >> 2, ak = (tid & 3) * E;
      const int gm = m0 + am;
      for (int u = 0; u < E; ++u) {
        const int gk = k0 + ak + u;
        ra[u] = (gm < d.M && gk < d.K) ? A[int64_t(gm) * d.sam + int64_t(gk) * d.sak] : T(0);
      }
    } else {
      const int ak = tid / TPR, am = (tid % TPR) * E;
      const int gk = k0 + ak;
      for (int u = 0; u < E; ++u) {
        const int gm = m0 + am + u;
        ra[u] = (gm < d.M && gk < d.K) ? A[int64_t(gm) * d.sam + int64_t(gk) * d.sak] : T(0);
      }
    }
    const int gk = k0 + bk;
    if (gk < d.K) {
      if (d.gidx) {
        const T* row = Cuser + int64_t(d.gidx[gk]) * ldcu + boff;
        for (int u = 0; u < E; ++u) {
          const int gn = n0 + bn + u;
          rb[u] = (gn < d.N && boff + gn < blim) ? row[gn] : T(0);
        }
      } else {
        const T* row = static_cast<const T*>(d.B) + int64_t(gk) * d.ldb;
        for (int u = 0; u < E; ++u) {
          const int gn = n0 + bn + u;
          rb[u] = (gn < d.N) ? row[gn] : T(0);
        }
      }
    } else {
      for (int u = 0; u < E; ++u) rb[u] = T(0);
    }
  };
  auto store = [&]() {
    if (A_KCONTIG) {
      const int am = tid >> 2, ak = (tid & 3) * E;
      for (int u = 0; u < E; ++u) As[ak + u][am] = ra[u];
    } else {
      const int ak = tid / TPR, am = (tid % TPR) * E;
      for (int u = 0; u < E; ++u) As[ak][am + u] = ra[u];
    }
    for (int u = 0; u < E; ++u) Bs[bk][bn + u] = rb[u];
  };

  load(0);
  for (int k0 = 0; k0 < d.K; k0 += KT) {
    store();
    __syncthreads();
    if (k0 + KT < d.K) load(k0 + KT);
    if constexpr (MODE == kModeBF16x6) {
      const int kb = 8 * (lane >> 4);
      bf16x8 ah[2], am[2], al[2], bh[2], bm[2], bl[2];
      for (int i = 0; i < 2; ++i) {
        float x[8];
        for (int e = 0; e < 8; ++e) x[e] = As[kb + e][wm + i * 16 + (lane & 15)];
        split8x3(x, ah[i], am[i], al[i]);
      }
      for (int j = 0; j < 2; ++j) {
        float x[8];
        for (int e = 0; e < 8; ++e) x[e] = Bs[kb + e][wn + j * 16 + (lane & 15)];
        split8x3(x, bh[j], bm[j], bl[j]);
      }
      for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j) {   // smallest terms first
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(am[i], bm[j], acc[i][j], 0, 0, 0);
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[i], bh[j], acc[i][j], 0, 0, 0);
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[i], bl[j], acc[i][j], 0, 0, 0);
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(am[i], bh[j], acc[i][j], 0, 0, 0);
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[i], bm[j], acc[i][j], 0, 0, 0);
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[i], bh[j], acc[i][j], 0, 0, 0);
        }
    } else if constexpr (MODE == kModeBF16x3) {
      const int kb = 8 * (lane >> 4);
      bf16x8 ah[2], al[2], bh[2], bl[2];
      for (int i = 0; i < 2; ++i) {
        float x[8];
        for (int e = 0; e < 8; ++e) x[e] = As[kb + e][wm + i * 16 + (lane & 15)];
        split8(x, ah[i], al[i]);
      }
      for (int j = 0; j < 2; ++j) {
        float x[8];
        for (int e = 0; e < 8; ++e) x[e] = Bs[kb + e][wn + j * 16 + (lane & 15)];
        split8(x, bh[j], bl[j]);
      }
      for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j) {
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[i], bh[j], acc[i][j], 0, 0, 0);
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[i], bl[j], acc[i][j], 0, 0, 0);
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[i], bh[j], acc[i][j], 0, 0, 0);
        }
    } else {
#pragma unroll
      for (int kk = 0; kk < KT; kk += 4) {
        const int kr = kk + (lane >> 4);
        T a[2], b[2];
        for (int i = 0; i < 2; ++i) a[i] = As[kr][wm + i * 16 + (lane & 15)];
        for (int j = 0; j < 2; ++j) b[j] = Bs[kr][wn + j * 16 + (lane & 15)];
        for (int i = 0; i < 2; ++i)
          for (int j = 0; j < 2; ++j) acc[i][j] = mfma4(a[i], b[j], acc[i][j]);
      }
    }
    __syncthreads();
    if constexpr (kFlush) {
      if (++ktile == FLUSH) {
        ktile = 0;
        for (int i = 0; i < 2; ++i)
          for (int j = 0; j < 2; ++j) {
            for (int r = 0; r < 4; ++r) acc64[i][j][r] += double(acc[i][j][r]);
            acc[i][j] = Acc{};
          }
      }
    }
  }
  if constexpr (kFlush)
    for (int i = 0; i < 2; ++i)
      for (int j = 0; j < 2; ++j)
        for (int r = 0; r < 4; ++r) acc64[i][j][r] += double(acc[i][j][r]);
  OutT* Cout = static_cast<OutT*>(d.C);
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j) {
      const int col = n0 + wn + j * 16 + (lane & 15);
      if (col >= d.N) continue;
      for (int r = 0; r < 4; ++r) {
        const int row = m0 + wm + i * 16 + acc_row<Acc>(lane >> 4, r);
        if (row >= d.M) continue;
        OutT* c = Cout + int64_t(row) * d.ldc + col;
        OutT v;
        if constexpr (kFlush) v = OutT(acc64[i][j][r]);
        else v = OutT(acc[i][j][r]);
        *c = accumulate ? *c + v : v;
      }
    }
}

// --------------------------------------------------------------------------
// translation: out[t] = sum_{e in CSR(t)} T[op_e] * data[src_e]   (overwrite)
// Each box is Q rows x ncol columns.  Block = 4 waves x 64 columns; each wave
// holds MT 16-row tiles x 4 column tiles of accumulators.  Blocks are
// renumbered so that each XCD walks contiguous (column tile, target) ranges:
// neighbouring targets then share their sources in that XCD's L2.
// T = double: FP64 MFMA; T = float: FP32 MFMA.
// --------------------------------------------------------------------------
template <class T, int MT>
__global__ __launch_bounds__(256) void translate_kernel(T* __restrict__ data, int64_t box_stride, int64_t ncol,
                                                        int Q, int KS, const int32_t* __restrict__ tgt_box,
                                                        const int32_t* __restrict__ src_ptr,
                                                        const int32_t* __restrict__ src_box,
                                                        const int32_t* __restrict__ src_op,
                                                        const T* __restrict__ ops, int ntgt, int64_t nblocks) {
  using Acc = typename std::conditional<std::is_same<T, double>::value, d4, f4>::type;
  const int64_t per = (int64_t(gridDim.x) + 7) / 8;
  const int64_t logical = int64_t(blockIdx.x % 8) * per + blockIdx.x / 8;
  if (logical >= nblocks) return;
  const int t = int(logical % ntgt);
  const int64_t ct = logical / ntgt;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t colbase = ct * 256 + wave * 64;
  Acc acc[MT][4];
  for (int i = 0; i < MT; ++i)
    for (int j = 0; j < 4; ++j) acc[i][j] = Acc{};
  const int64_t opsz = int64_t(MT) * KS * 64;
  const int e0 = src_ptr[t], e1 = src_ptr[t + 1];
  for (int e = e0; e < e1; ++e) {
    const T* X = data + int64_t(src_box[e]) * box_stride;
    const T* Tm = ops + int64_t(src_op[e]) * opsz;
    for (int ks = 0; ks < KS; ++ks) {
      const int row = ks * 4 + (lane >> 4);
      T b[4];
      for (int j = 0; j < 4; ++j) {
        const int64_t col = colbase + j * 16 + (lane & 15);
        b[j] = (row < Q && col < ncol) ? X[int64_t(row) * ncol + col] : T(0);
      }
      for (int i = 0; i < MT; ++i) {
        const T a = Tm[(int64_t(i) * KS + ks) * 64 + lane];
        for (int j = 0; j < 4; ++j) acc[i][j] = mfma4(a, b[j], acc[i][j]);
      }
    }
  }
  T* Y = data + int64_t(tgt_box[t]) * box_stride;
  for (int i = 0; i < MT; ++i)
    for (int j = 0; j < 4; ++j) {
      const int64_t col = colbase + j * 16 + (lane & 15);
      if (col >= ncol) continue;
      for (int r = 0; r < 4; ++r) {
        const int row = i * 16 + acc_row<Acc>(lane >> 4, r);
        if (row < Q) Y[int64_t(row) * ncol + col] = T(acc[i][j][r]);
      }
    }
}

// out[r*ldo + c] = float(in[r*ldi + c]) for r < rows, c < cols
__global__ void to_float_kernel(const double* __restrict__ in, int64_t ldi, float* __restrict__ out, int64_t ldo,
                                int64_t rows, int64_t cols) {
  const int64_t n = rows * cols;
  for (int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; e < n; e += int64_t(gridDim.x) * blockDim.x) {
    const int64_t r = e / cols, c = e % cols;
    out[r * ldo + c] = float(in[r * ldi + c]);
  }
}

// K[r, i0 + i] = (acc ? K : 0) + sum_{e in occ(r)} KB[row_e, i]   (fixed order)
__global__ __launch_bounds__(256) void reduce_kernel(const double* __restrict__ KB, int64_t ni,
                                                     const int32_t* __restrict__ occ_ptr,
                                                     const int32_t* __restrict__ occ_row, double* __restrict__ K,
                                                     int64_t ldk, int i0, int accumulate) {
  const int r = blockIdx.y;
  const int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (i >= ni) return;
  double s = 0.0;
  for (int e = occ_ptr[r]; e < occ_ptr[r + 1]; ++e) s += KB[int64_t(occ_row[e]) * ni + i];
  double* k = K + int64_t(r) * ldk + i0 + i;
  *k = accumulate ? *k + s : s;
}

__global__ void zero_cols_kernel(double* __restrict__ K, int64_t ldk, int i0, int64_t ni) {
  const int r = blockIdx.y;
  const int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (i < ni) K[int64_t(r) * ldk + i0 + i] = 0.0;
}

// --------------------------------------------------------------------------
// host orchestration
// --------------------------------------------------------------------------
template <class T>
struct DevBuf {
  T* p = nullptr;
  size_t n = 0;
  void free() {
    if (p) (void)hipFree(p);
    p = nullptr;
    n = 0;
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

struct Pass {           // one translation launch
  int ntgt = 0;
  DevBuf<int32_t> tgt_box, src_ptr, src_box, src_op;
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
  std::vector<Pass> up, down;     // up[k]: level depth-1-k ; down[k]: level lmin+k
  DevBuf<int32_t> occ_ptr, occ_row;
  int nbox = 0;                    // boxes on levels lmin..depth
  std::vector<int32_t> leaf_box;   // leaf -> box slot
  // per workspace shape (j batch, n_i, precision)
  int ws_jb = -1, ws_ni = -1, ws_prec = -1;
  DevBuf<char> H, data;           // element type of the precision (double / float)
  DevBuf<double> KB;              // per-leaf K partials, always FP64
  DevBuf<float> Cf;               // FP32 copy of C for the mixed paths
  DevBuf<GemmDesc> d_half, d_omega, d_l2p;
  DevBuf<GemmTile> t_half, t_omega, t_l2p;
  int n_half = 0, n_omega = 0, n_l2p = 0;
  size_t bytes = 0;
  // profiling: (class, start, end) event pairs recorded on the call's stream
  std::vector<hipEvent_t> ev_pool;
  size_t ev_used = 0;
  std::vector<int> ev_class;
  std::vector<int64_t> launches;
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
  ~ProfScope() {
    if (!ds) return;
    (void)hipEventRecord(ds->ev_pool[idx + 1], st);
    ds->ev_class.push_back(cls);
    if (ds->launches.size() < OCCK_K_NCLASS) ds->launches.assign(OCCK_K_NCLASS, 0);
    ds->launches[cls] += nlaunch;
  }
};

static size_t device_cap() {
  const char* s = std::getenv("OCCK_MAX_DEVICE_BYTES");
  if (s && *s) return size_t(std::strtoull(s, nullptr, 10));
  return size_t(96) << 30;
}

static void free_state(DeviceState* ds);

static void upload_tree_into(Tree* t, DeviceState* ds);

static void upload_tree(Tree* t) {
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
    ps.tgt_box.upload(tb);
    ps.src_ptr.upload(sp);
    ps.src_box.upload(sb);
    ps.src_op.upload(so);
    ds->up.push_back(std::move(ps));
  }
  // downward passes: Mloc targets at lev; sources = parent Mloc (L2L) + IL Omega (M2L)
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
    ps.tgt_box.upload(tb);
    ps.src_ptr.upload(sp);
    ps.src_box.upload(sb);
    ps.src_op.upload(so);
    ds->down.push_back(std::move(ps));
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

static void tiles_for(std::vector<GemmTile>& tiles, int prob, int M, int N) {
  for (int mt = 0; mt < (M + 63) / 64; ++mt)
    for (int nt = 0; nt < (N + 63) / 64; ++nt) tiles.push_back({prob, mt, nt, 0});
}

static void setup_workspace(Tree* t, int jb, int ni, int prec) {
  DeviceState* ds = t->dev;
  if (ds->ws_jb == jb && ds->ws_ni == ni && ds->ws_prec == prec) return;
  const int Q = t->Q, nl = t->nleaf();
  const size_t es = prec == OCCK_PREC_FP64 ? 8 : 4;
  const int64_t sum_nb = ds->f_off[nl];
  const int64_t ncol = int64_t(jb) * ni;
  const size_t need = size_t(sum_nb) * Q * jb * es + size_t(2) * ds->nbox * Q * size_t(ncol) * es +
                      size_t(sum_nb) * ni * 8;
  if (need + ds->bytes > device_cap()) throw std::bad_alloc();
  ds->ws_jb = -1;   // invalid until every buffer and descriptor is in place
  ds->ws_ni = -1;
  ds->ws_prec = -1;
  ds->H.free();
  ds->data.free();
  ds->KB.free();
  ds->H.alloc(size_t(sum_nb) * Q * jb * es);
  ds->data.alloc(size_t(2) * ds->nbox * Q * size_t(ncol) * es);
  ds->KB.alloc(size_t(sum_nb) * ni);
  const int64_t box_stride = int64_t(Q) * ncol;
  const char* Obase = prec == OCCK_PREC_FP64 ? reinterpret_cast<const char*>(ds->O.p)
                                             : reinterpret_cast<const char*>(ds->Of.p);
  std::vector<GemmDesc> dh, dom, dl;
  std::vector<GemmTile> th, tom, tl2;
  for (int b = 0; b < nl; ++b) {
    const int nb = int(t->leaf_funcs[b].size());
    const int64_t hoff = ds->f_off[b] * Q * jb;   // H^B[t][q][j], ld Q*jb (elements)
    const int32_t* g = ds->funcs.p + ds->f_off[b];
    for (int q = 0; q < Q; ++q) {  // H_q = O^B_q C_B[:, J]
      GemmDesc d{};
      d.A = Obase + (ds->O_off[b] + int64_t(q) * nb * nb) * es;
      d.sam = nb;
      d.sak = 1;
      d.gidx = g;
      d.C = ds->H.p + (hoff + int64_t(q) * jb) * es;
      d.ldc = int64_t(Q) * jb;
      d.M = nb;
      d.N = jb;
      d.K = nb;
      tiles_for(th, int(dh.size()), d.M, d.N);
      dh.push_back(d);
    }
    {  // Omega[(q,j), i] = sum_t H[t][(q,j)] C[f(t), i0+i]
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
    {  // KB[r, i] (+)= sum_(q,j) H[r][(q,j)] Mloc[(q,j), i]
      GemmDesc d{};
      d.A = ds->H.p + hoff * es;
      d.sam = int64_t(Q) * jb;
      d.sak = 1;
      d.B = ds->data.p + int64_t(ds->nbox + ds->leaf_box[b]) * box_stride * es;
      d.ldb = ni;
      d.C = ds->KB.p + ds->f_off[b] * ni;
      d.ldc = ni;
      d.M = nb;
      d.N = ni;
      d.K = Q * jb;
      tiles_for(tl2, int(dl.size()), d.M, d.N);
      dl.push_back(d);
    }
  }
  ds->d_half.upload(dh);
  ds->t_half.upload(th);
  ds->d_omega.upload(dom);
  ds->t_omega.upload(tom);
  ds->d_l2p.upload(dl);
  ds->t_l2p.upload(tl2);
  ds->n_half = int(th.size());
  ds->n_omega = int(tom.size());
  ds->n_l2p = int(tl2.size());
  ds->ws_jb = jb;
  ds->ws_ni = ni;
  ds->ws_prec = prec;
}

template <class T>
static void launch_translate(const Tree* t, const Pass& ps, T* data, int64_t box_stride, int64_t ncol, const T* ops,
                             hipStream_t st) {
  const int Q = t->Q, KS = ksteps_of(Q);
  const int64_t nct = (ncol + 255) / 256;
  const int64_t nblocks = nct * ps.ntgt;
  const int64_t grid = ((nblocks + 7) / 8) * 8;
  if (grid > 0x7fffffff) throw std::invalid_argument("translation grid too large; lower jblock");
#define OCCK_TR(MT)                                                                                           \
  hipLaunchKernelGGL((translate_kernel<T, MT>), dim3(unsigned(grid)), dim3(256), 0, st, data, box_stride, ncol, \
                     Q, KS, ps.tgt_box.p, ps.src_ptr.p, ps.src_box.p, ps.src_op.p, ops, ps.ntgt, nblocks)
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

static void launch_to_float(const double* in, int64_t ldi, float* out, int64_t ldo, int64_t rows, int64_t cols,
                            hipStream_t st) {
  const int64_t n = rows * cols;
  const int64_t blocks = std::min<int64_t>((n + 255) / 256, 65536);
  if (n == 0) return;
  hipLaunchKernelGGL(to_float_kernel, dim3(unsigned(blocks)), dim3(256), 0, st, in, ldi, out, ldo, rows, cols);
  HIP_OK(hipGetLastError());
}

void device_free(Tree* t) {
  if (t->dev) free_state(t->dev);
  t->dev = nullptr;
}

static void free_state(DeviceState* ds) {
  for (hipEvent_t e : ds->ev_pool) (void)hipEventDestroy(e);
  ds->ev_pool.clear();
  ds->Of.free();
  ds->opsf.free();
  ds->Cf.free();
  ds->O.free();
  ds->funcs.free();
  ds->opparam.free();
  ds->ops.free();
  for (auto& p : ds->up) { p.tgt_box.free(); p.src_ptr.free(); p.src_box.free(); p.src_op.free(); }
  for (auto& p : ds->down) { p.tgt_box.free(); p.src_ptr.free(); p.src_box.free(); p.src_op.free(); }
  ds->occ_ptr.free();
  ds->occ_row.free();
  ds->H.free();
  ds->data.free();
  ds->KB.free();
  ds->d_half.free(); ds->d_omega.free(); ds->d_l2p.free();
  ds->t_half.free(); ds->t_omega.free(); ds->t_l2p.free();
  delete ds;
}

static int auto_jblock(const Tree* t, int nj, int ni, size_t es) {
  const size_t cap = device_cap();
  const int Q = t->Q;
  int64_t sum_nb = 0;
  for (const auto& f : t->leaf_funcs) sum_nb += int64_t(f.size());
  int64_t nbox = 0;
  for (int lev = t->lmin; lev <= t->params.depth; ++lev) nbox += int64_t(t->boxes[lev].size());
  const size_t budget = std::min(cap / 2, size_t(32) << 30);
  int jb = std::min(nj, 256);
  while (jb > 1) {
    const size_t need = size_t(sum_nb) * Q * jb * es + size_t(2) * nbox * Q * size_t(jb) * ni * es;
    if (need <= budget) break;
    jb = (jb + 1) / 2;
  }
  return std::max(1, jb);
}

// One j batch: half transform, Omega, upward, downward, L2P.
template <int MODE>
static void run_batches(Tree* t, DeviceState* ds, const typename ModeT<MODE>::T* Cg, int64_t ldcg, int i0, int i1,
                        int j0, int j1, int jb, int ni, bool prof, hipStream_t st) {
  using T = typename ModeT<MODE>::T;
  const int Q = t->Q;
  const int64_t ncol = int64_t(jb) * ni;
  const int64_t box_stride = int64_t(Q) * ncol;
  T* data = reinterpret_cast<T*>(ds->data.p);
  const T* ops = MODE == kModeF64 ? reinterpret_cast<const T*>(ds->ops.p) : reinterpret_cast<const T*>(ds->opsf.p);
  const int nj = j1 - j0;
  const int nblk = (nj + jb - 1) / jb;
  for (int kb = 0; kb < nblk; ++kb) {
    const int64_t jstart = j0 + int64_t(kb) * jb;
    {
      ProfScope ps(ds, prof, OCCK_K_HALF, st);
      hipLaunchKernelGGL((gemm_kernel<MODE, true, T>), dim3(unsigned(ds->n_half)), dim3(256), 0, st, ds->d_half.p,
                         ds->t_half.p, Cg, ldcg, jstart, int64_t(j1), 0);
    }
    {
      ProfScope ps(ds, prof, OCCK_K_OMEGA, st);
      hipLaunchKernelGGL((gemm_kernel<MODE, false, T>), dim3(unsigned(ds->n_omega)), dim3(256), 0, st,
                         ds->d_omega.p, ds->t_omega.p, Cg, ldcg, int64_t(i0), int64_t(i1), 0);
    }
    {
      ProfScope ps(ds, prof, OCCK_K_UP, st, int(ds->up.size()));
      for (const Pass& p : ds->up) launch_translate<T>(t, p, data, box_stride, ncol, ops, st);
    }
    {
      ProfScope ps(ds, prof, OCCK_K_DOWN, st, int(ds->down.size()));
      for (const Pass& p : ds->down) launch_translate<T>(t, p, data, box_stride, ncol, ops, st);
    }
    {
      ProfScope ps(ds, prof, OCCK_K_L2P, st);
      hipLaunchKernelGGL((gemm_kernel<MODE, true, double>), dim3(unsigned(ds->n_l2p)), dim3(256), 0, st,
                         ds->d_l2p.p, ds->t_l2p.p, Cg, ldcg, int64_t(0), int64_t(0), kb > 0 ? 1 : 0);
    }
    HIP_OK(hipGetLastError());
  }
}

int32_t far_K(Tree* t, const double* C, int64_t ldc, int32_t nocc, int32_t i0, int32_t i1, int32_t j0,
              int32_t j1, const occk_far_opts* opts, double* K, int64_t ldk, void* stream) {
  if (opts->rank_mode != OCCK_RANK_FIXED) {
    set_error("occk_far_K: learned ranks are not built in this library version");
    return OCCK_ESTATE;
  }
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
    if (!t->dev) upload_tree(t);
    DeviceState* ds = t->dev;
    if (mixed && !ds->Of.p) {   // FP32 copies of the per-tree operands (once)
      ds->Of.alloc(ds->O.n);
      ds->opsf.alloc(ds->ops.n);
      launch_to_float(ds->O.p, 0, ds->Of.p, 0, 1, int64_t(ds->O.n), st);
    }
    const size_t es = mixed ? 4 : 8;
    const int jb = opts->jblock > 0 ? std::min<int>(opts->jblock, nj) : auto_jblock(t, nj, ni, es);
    setup_workspace(t, jb, ni, prec);
    const int Q = t->Q;
    const bool prof = t->profile != 0;
    {
      ProfScope ps(ds, prof, OCCK_K_OPGEN, st);
      hipLaunchKernelGGL(opgen_kernel, dim3(unsigned(t->ops.size())), dim3(64), 0, st, ds->opparam.p, ds->ops.p,
                         t->L, Q);
      HIP_OK(hipGetLastError());
    }
    if (mixed) {
      ProfScope ps(ds, prof, OCCK_K_CONVERT, st, 2);
      launch_to_float(ds->ops.p, 0, ds->opsf.p, 0, 1, int64_t(ds->ops.n), st);
      ds->Cf.alloc(size_t(nbasis) * nocc);
      launch_to_float(C, ldc, ds->Cf.p, nocc, nbasis, nocc, st);
    }
    if (prec == OCCK_PREC_FP64)
      run_batches<kModeF64>(t, ds, C, ldc, i0, i1, j0, j1, jb, ni, prof, st);
    else if (prec == OCCK_PREC_FP32)
      run_batches<kModeF32>(t, ds, ds->Cf.p, nocc, i0, i1, j0, j1, jb, ni, prof, st);
    else if (prec == OCCK_PREC_BF16X3)
      run_batches<kModeBF16x3>(t, ds, ds->Cf.p, nocc, i0, i1, j0, j1, jb, ni, prof, st);
    else
      run_batches<kModeBF16x6>(t, ds, ds->Cf.p, nocc, i0, i1, j0, j1, jb, ni, prof, st);
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
      HIP_OK(hipEventSynchronize(ds->ev_pool[2 * k + 1]));
      float e = 0.f;
      HIP_OK(hipEventElapsedTime(&e, ds->ev_pool[2 * k], ds->ev_pool[2 * k + 1]));
      if (ms) ms[ds->ev_class[k]] += double(e);
    }
    if (launches && !ds->launches.empty())
      for (int c = 0; c < OCCK_K_NCLASS; ++c) launches[c] = ds->launches[c];
  } catch (const HipError& e) {
    set_error(e.what());
    return OCCK_EHIP;
  }
  ds->ev_class.clear();
  ds->ev_used = 0;
  ds->launches.assign(OCCK_K_NCLASS, 0);
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
