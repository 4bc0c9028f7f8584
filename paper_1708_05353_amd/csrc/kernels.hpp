// Device code of the far-field exchange: descriptors, FP64 operator
// generation, tile-level GEMM and translation routines (shared by the
// per-stage kernels and the persistent batched kernel), reductions.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>

#include "occk_internal.hpp"

typedef double d4 __attribute__((ext_vector_type(4)));

namespace occk {

// Global-memory view of a pointer.  Pointers read from device tables (the
// persistent batched kernel) are generic to the compiler, which then emits
// flat loads and stores; the tile routines below access every operand
// through this view so that they compile to global loads and stores.
template <class T>
using gbl = __attribute__((address_space(1))) T;
template <class T>
__device__ __forceinline__ gbl<T>* as_global(T* p) {
  return (gbl<T>*)p;
}
// Streaming store (non-temporal): for results that the next pass reads
// long after the L2 has cycled through other data.
template <class T>
__device__ __forceinline__ void store_stream(gbl<T>* p, T v) {
  __builtin_nontemporal_store(v, p);
}
// Read-only view for tables and operators that no kernel writes while the
// reading kernel runs (CSR lists, descriptors, operators): wave-uniform
// loads through it compile to scalar loads.
template <class T>
using cst = __attribute__((address_space(4))) T;
template <class T>
__device__ __forceinline__ const cst<T>* as_const(const T* p) {
  return (const cst<T>*)p;
}
// Copy of a table entry (a descriptor struct) read through the read-only view.
template <class S>
__device__ __forceinline__ S load_const(const S* p) {
  static_assert(sizeof(S) % 4 == 0, "whole dwords");
  S out;
  const cst<uint32_t>* src = (const cst<uint32_t>*)p;
  uint32_t* dst = reinterpret_cast<uint32_t*>(&out);
  for (int i = 0; i < int(sizeof(S) / 4); ++i) dst[i] = src[i];
  return out;
}

// --------------------------------------------------------------------------
// device-side descriptors
// --------------------------------------------------------------------------
struct GemmDesc {       // element types follow the kernel's mode (output: OutT)
  const void* A;       // A(m,k) = A[m*sam + k*sak]
  int64_t sam, sak;
  const void* B;       // B(k,n) = B[k*ldb + n]                (gidx == nullptr)
  int64_t ldb;
  const int32_t* gidx; // B(k,n) = Cuser[gidx[k]*ldcu + boff + n] (gather from C)
  void* C;             // C(m,n) = C[m*ldc + n*ldcn]   (ldcn 0 means 1)
  int64_t ldc, ldcn;
  // K segments: the contraction runs over nseg (0 means 1) segments of K
  // terms; segment s reads A + s*sa_seg and B + s*sb_seg (plain B only).
  int64_t sa_seg, sb_seg;
  int32_t M, N, K, nseg;
};
// Per-launch parameters shared by every tile of one grouped GEMM launch.
struct GemmRun {
  int64_t boff, blim;  // gathered B: column offset into Cuser, columns at or beyond blim read as 0
  int64_t koff;        // every segment contracts k in [koff, K)
  int64_t coff;        // output pointer offset (elements)
  int32_t nlo;         // output columns below nlo are not written
  int32_t mlim;        // rows at or beyond mlim are neither read from A (zero) nor written (0: no limit)
  int32_t accumulate;  // C += A B instead of C = A B
  int32_t tile0;       // the launch computes tiles [tile0, tile0 + ntiles)
  int32_t ntiles;
  int32_t nhi;         // output columns at or beyond nhi are not written, tiles starting there skipped (0: none)
  int32_t klim;        // k runs over [koff, min(K, klim)) (0: K)
  int32_t amoff;       // A is read at row m + amoff (the rows of B and C are not shifted)
  int32_t akoff;       // A is read at column k + akoff (the k of B is not shifted)
  int64_t aptr, bptr;  // element offsets added to the A and (plain) B pointers of every problem
};
struct GemmTile {
  int32_t prob, mt, nt, pad;
};
// Columns carried by the translations of one j batch.  Box data are Q rows
// of ncol = jb*ni columns, column (j, i) at j*ni + i.  Only columns with
// i >= istart are carried (the symmetric schedule starts i at the batch's
// first j); nvalid = jb*(ni - istart) of them, numbered v = j*(ni - istart)
// + (i - istart).
// With occupied-pair screening the carried i of a batch end at iend (0: ni),
// nvalid = jb*(iend - istart), v = j*(iend - istart) + (i - istart).
struct ColMap {
  int64_t ncol, ni, istart, nvalid, iend;
};
__host__ __device__ inline int64_t carried_col(const ColMap& cm, int64_t v) {
  if (cm.istart == 0 && cm.iend == 0) return v;
  const int64_t nk = (cm.iend > 0 ? cm.iend : cm.ni) - cm.istart;
  const int64_t j = v / nk;
  return j * cm.ni + cm.istart + (v - j * nk);
}
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
static __device__ void regular_table(int L, const double* v, Cplx* tab) {
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
static __device__ void irregular_table(int L, const double* v, Cplx* tab) {
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
static __device__ double real_entry(int type, const Cplx* tab, int row, int col) {
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

// ops layout ("fragment order" of the FP64/FP32 MFMA A operand): element
// ((mt*KS + ks)*64 + lane) holds T[mt*16 + lane%16][ks*4 + lane/16].
// Generates one operator with nthreads threads (thread index tid); tab is a
// shared table of at least (2L+1)(2L+2)/2 entries.  The FP64 result is also
// written rounded to FP32 when outf is non-null.
// perm (may be null): entry (row, col) of the generated matrix is
// T[perm[row]][perm[col]] (the components in the order perm lists them).
static __device__ void opgen_one(const OpParam& p, double* out, float* outf, int L, int Q, Cplx* tab, int tid,
                          int nthreads, const int32_t* perm = nullptr) {
  if (tid == 0) {
    if (p.type == kOpM2L) irregular_table(2 * L, p.d, tab);
    else regular_table(L, p.d, tab);
  }
  __syncthreads();
  const int MT = mtiles_of(Q), KS = ksteps_of(Q);
  for (int e = tid; e < MT * KS * 64; e += nthreads) {
    const int lane = e & 63;
    const int frag = e >> 6;
    const int mt = frag / KS, ks = frag % KS;
    const int row = mt * 16 + (lane & 15), col = ks * 4 + (lane >> 4);
    double v = 0.0;
    if (row < Q && col < Q) {
      const int r = perm ? perm[row] : row, c = perm ? perm[col] : col;
      v = real_entry(p.type, tab, r, c);
      if (p.weighted) v *= l2p_weight(r);
    }
    if (out) as_global(out)[e] = v;
    if (outf) as_global(outf)[e] = float(v);
  }
  __syncthreads();
}

static __global__ __launch_bounds__(64) void opgen_kernel(const OpParam* __restrict__ params, double* __restrict__ ops,
                                                   int L, int Q) {
  __shared__ Cplx tab[(2 * kMaxL + 1) * (2 * kMaxL + 2) / 2];
  const int64_t sz = int64_t(mtiles_of(Q)) * ksteps_of(Q) * 64;
  opgen_one(params[blockIdx.x], ops + int64_t(blockIdx.x) * sz, nullptr, L, Q, tab, threadIdx.x, 64);
}

// The same operators with their components reordered by perm (the MFMA
// translations of axis-aligned trees, whose structural zeros then form
// whole blocks).
static __global__ __launch_bounds__(64) void opgen_perm_kernel(const OpParam* __restrict__ params,
                                                        double* __restrict__ ops, int L, int Q,
                                                        const int32_t* __restrict__ perm) {
  __shared__ Cplx tab[(2 * kMaxL + 1) * (2 * kMaxL + 2) / 2];
  const int64_t sz = int64_t(mtiles_of(Q)) * ksteps_of(Q) * 64;
  opgen_one(params[blockIdx.x], ops + int64_t(blockIdx.x) * sz, nullptr, L, Q, tab, threadIdx.x, 64, perm);
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

// The splits round to nearest even with the hardware's packed conversion
// (two FP32 values to two bf16 per instruction); a bf16 value widens back to
// FP32 exactly as its bits shifted into the high half.
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef float f2 __attribute__((ext_vector_type(2)));
__device__ inline f2 widen2(bf16x2 v) {
  const uint32_t u = __builtin_bit_cast(uint32_t, v);
  return f2{__uint_as_float(u << 16), __uint_as_float(u & 0xffff0000u)};
}

// x[e] -> hi[e] + lo[e] as bf16 vectors
__device__ inline void split8(const float* x, bf16x8& hi, bf16x8& lo) {
  bf16x2 h[4], l[4];
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const f2 v{x[2 * e], x[2 * e + 1]};
    h[e] = __builtin_convertvector(v, bf16x2);
    l[e] = __builtin_convertvector(v - widen2(h[e]), bf16x2);
  }
  hi = __builtin_shufflevector(__builtin_shufflevector(h[0], h[1], 0, 1, 2, 3),
                               __builtin_shufflevector(h[2], h[3], 0, 1, 2, 3), 0, 1, 2, 3, 4, 5, 6, 7);
  lo = __builtin_shufflevector(__builtin_shufflevector(l[0], l[1], 0, 1, 2, 3),
                               __builtin_shufflevector(l[2], l[3], 0, 1, 2, 3), 0, 1, 2, 3, 4, 5, 6, 7);
}

// x[e] -> hi[e] + mid[e] + lo[e] as bf16 vectors
__device__ inline void split8x3(const float* x, bf16x8& hi, bf16x8& mid, bf16x8& lo) {
  bf16x2 h[4], m[4], l[4];
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const f2 v{x[2 * e], x[2 * e + 1]};
    h[e] = __builtin_convertvector(v, bf16x2);
    const f2 r1 = v - widen2(h[e]);
    m[e] = __builtin_convertvector(r1, bf16x2);
    l[e] = __builtin_convertvector(r1 - widen2(m[e]), bf16x2);
  }
  hi = __builtin_shufflevector(__builtin_shufflevector(h[0], h[1], 0, 1, 2, 3),
                               __builtin_shufflevector(h[2], h[3], 0, 1, 2, 3), 0, 1, 2, 3, 4, 5, 6, 7);
  mid = __builtin_shufflevector(__builtin_shufflevector(m[0], m[1], 0, 1, 2, 3),
                                __builtin_shufflevector(m[2], m[3], 0, 1, 2, 3), 0, 1, 2, 3, 4, 5, 6, 7);
  lo = __builtin_shufflevector(__builtin_shufflevector(l[0], l[1], 0, 1, 2, 3),
                               __builtin_shufflevector(l[2], l[3], 0, 1, 2, 3), 0, 1, 2, 3, 4, 5, 6, 7);
}

__device__ inline d4 mfma4(double a, double b, d4 c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }
__device__ inline f4 mfma4(float a, float b, f4 c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }

// output row of accumulator element r for lane group g = lane/16 inside a 16-row tile
template <class Acc> __device__ inline int acc_row(int g, int r);
template <> __device__ inline int acc_row<d4>(int g, int r) { return g + 4 * r; }
template <> __device__ inline int acc_row<f4>(int g, int r) { return 4 * g + r; }

// --------------------------------------------------------------------------
// grouped GEMM: C(m,n) (+)= sum_k A(m,k) B(k,n) over a list of problems.
// One 256-thread block computes one BM x BN output tile; the 4 waves form a
// WGM x WGN grid, each wave TM x TN MFMA 16x16 tiles.  K is staged through
// LDS in steps of KT with the next step's global loads in flight during the
// current step's MFMAs.
//   GemmSquare 64 x 64  (2 x 2 waves of 2 x 2 tiles)
//   GemmRows48 48 x 64  (1 x 4 waves of 3 x 1 tiles): a leaf's n_B rows
//              (typically 80..144) padded to a multiple of 48, not 64
//   GemmCols48 64 x 48  (4 x 1 waves of 1 x 3 tiles): the transpose case
//   GemmCols144 64 x 144 (4 x 1 waves of 1 x 9 tiles): the transpose case
//              with the n_B <= 144 columns of a leaf in one tile
//   GemmRows144 144 x 64 (1 x 4 waves of 9 x 1 tiles): the n_B <= 144 rows
//              of a leaf in one tile
// --------------------------------------------------------------------------
template <int WGM_, int WGN_, int TM_, int TN_>
struct GemmShape {
  static_assert(WGM_ * WGN_ == 4, "four waves");
  static constexpr int WGM = WGM_, WGN = WGN_, TM = TM_, TN = TN_;
  static constexpr int BM = WGM * TM * 16, BN = WGN * TN * 16;
};
using GemmSquare = GemmShape<2, 2, 2, 2>;
using GemmRows48 = GemmShape<1, 4, 3, 1>;   // 48 x 64: the n_B rows of a leaf in tiles of 48
using GemmCols48 = GemmShape<4, 1, 1, 3>;   // 64 x 48: the transpose case
using GemmCols144 = GemmShape<4, 1, 1, 9>;  // 64 x 144: the transpose case, a whole leaf per tile
using GemmRows144 = GemmShape<1, 4, 9, 1>;  // 144 x 64: a whole leaf per tile

// NB = 2: double-buffered operand tiles (one barrier per K tile); NB = 1:
// single buffer (two barriers per K tile, half the LDS).
template <int MODE, class S, int NB>
struct GemmSmemPlain {
  typename ModeT<MODE>::T A[NB][ModeT<MODE>::KT][S::BM + 1];
  typename ModeT<MODE>::T B[NB][ModeT<MODE>::KT][S::BN + 1];
};
// Split-BF16 modes: the operand tiles are split once, when they are stored,
// and held as NP bf16 planes in the MFMA fragment layout: row m of A (column
// n of B) holds its KT = 32 k as four 8-element chunks, one 16-byte fragment
// each.  Chunk g of row m sits at position split_chunk(m, g): with 64-byte
// rows, the 16-byte accesses of 8 (or 16) consecutive rows at one chunk then
// fall on distinct banks of a 32 (or 64) bank LDS.
constexpr bool mode_split(int mode) { return mode == kModeBF16x3 || mode == kModeBF16x6; }
constexpr int mode_planes(int mode) { return mode == kModeBF16x6 ? 3 : 2; }
__device__ inline int split_chunk(int m, int g) { return g ^ (((m >> 1) ^ (m >> 2)) & 3); }
template <class S, int NB, int NP>
struct GemmSmemSplit {
  bf16x8 A[NB][NP][S::BM][4];
  bf16x8 B[NB][NP][S::BN][4];
};
template <int MODE, class S = GemmSquare, int NB = 1>
using GemmSmem = typename std::conditional<mode_split(MODE), GemmSmemSplit<S, NB, mode_planes(MODE)>,
                                           GemmSmemPlain<MODE, S, NB>>::type;

// Read in place of operand elements outside their matrix: the GEMM operand
// loads take no branch and their values need no masking afterwards.
__device__ const double gemm_zero[2] = {0.0, 0.0};

template <int MODE, bool A_KCONTIG, bool GATHER, class OutT, class S = GemmSquare, int NB = 1, int DEPTH = 1>
__device__ void gemm_tile(const GemmDesc& d, int mt, int nt, const typename ModeT<MODE>::T* __restrict__ Cuser,
                          int64_t ldcu, const GemmRun& run, GemmSmem<MODE, S, NB>& sm) {
  using T = typename ModeT<MODE>::T;
  using Acc = typename ModeT<MODE>::Acc;
  constexpr int KT = ModeT<MODE>::KT;
  constexpr int BM = S::BM, BN = S::BN, TM = S::TM, TN = S::TN;
  constexpr int EA = BM * KT / 256, EB = BN * KT / 256;   // elements per thread per operand tile
  const int64_t boff = run.boff, blim = run.blim, koff = run.koff;   // koff < 2^31
  const int m0 = mt * BM, n0 = nt * BN;
  if (run.nhi > 0 && n0 >= run.nhi) return;   // the whole tile lies past the written columns (uniform)
  const int kend = run.klim > 0 && run.klim < d.K ? run.klim : d.K;   // k runs over [koff, kend) in every segment
  const int64_t kseg = int64_t(kend) - koff;                // terms per segment
  const int nseg = d.nseg > 0 ? d.nseg : 1;
  const int kpseg = kseg > 0 ? int((kseg + KT - 1) / KT) : 0;  // K tiles per segment
  const int nsteps = nseg * kpseg;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = (wave % S::WGM) * TM * 16, wn = (wave / S::WGM) * TN * 16;
  Acc acc[TM][TN];
  for (int i = 0; i < TM; ++i)
    for (int j = 0; j < TN; ++j) acc[i][j] = Acc{};
  // FP32 accumulators feeding an FP64 output are flushed into FP64 registers
  // every FLUSH K tiles, so FP32 rounding accumulates over at most FLUSH*KT =
  // 128 terms in every mixed mode.
  constexpr bool kFlush = std::is_same<OutT, double>::value && MODE != kModeF64;
  constexpr int FLUSH = 128 / KT;
  double acc64[kFlush ? TM : 1][kFlush ? TN : 1][kFlush ? 4 : 1];
  if constexpr (kFlush)
    for (int i = 0; i < TM; ++i)
      for (int j = 0; j < TN; ++j)
        for (int r = 0; r < 4; ++r) acc64[i][j][r] = 0.0;
  int ktile = 0;
  // DEPTH = 2 (with NB = 2): two register sets, the loads run two K tiles
  // ahead of the MFMAs
  static_assert(DEPTH == 1 || (DEPTH == 2 && NB == 2), "two-deep loads need two LDS buffers");
  constexpr int NR = DEPTH;
  constexpr bool kSplit = mode_split(MODE);
  T ra[NR][kSplit ? 1 : EA], rb[NR][kSplit ? 1 : EB];
  // Split-BF16 modes move whole k chunks: unit c = tid + 256 p of the A tile
  // is row m, chunk g (k = 8g .. 8g + 7), with m = c / KC, g = c % KC when A
  // is k-contiguous and m = c % BM, g = c / BM otherwise, so that the lanes
  // of a wave read adjacent memory; unit c of the B tile is column c % BN,
  // chunk c / BN.  Units past the tile (c >= BM KC) are whole waves.
  constexpr int KC = KT / 8;
  constexpr int UA = kSplit ? (BM * KC + 255) / 256 : 1, UB = kSplit ? (BN * KC + 255) / 256 : 1;
  float sa[kSplit ? NR : 1][UA][8], sb[kSplit ? NR : 1][UB][8];
  // Thread -> element maps of the operand tiles (element u of the thread):
  //   A k-contiguous: EA consecutive k of row am;
  //   A k-contiguous, KT not a multiple of EA (tiles of 48 rows, A_ROWS):
  //     column ak = tid % KT of rows am + u * (256 / KT);
  //   A m-contiguous, 64-wide tile (A_MW): element am = tid % 64 of k rows
  //     ak + u * 4, so that a wave loads and stores whole 64-element rows
  //     (coalesced loads, LDS stores without bank conflicts);
  //   A m-contiguous otherwise: EA consecutive m at k row ak;
  //   B, 64-wide tile (B_W): element bn = tid % 64 of k rows bk + u * 4;
  //   B otherwise: EB consecutive n at k row bk.
  constexpr bool A_ROWS = A_KCONTIG && (KT % EA != 0);
  constexpr bool A_MW = !A_KCONTIG && BM == 64;
  constexpr bool B_W = BN == 64;
  constexpr int ARW = 256 / 64;   // k rows per pass of the A_MW and B_W maps
  constexpr int TPRA = A_ROWS ? KT : (A_KCONTIG ? KT / EA : BM / EA), TPRB = BN / EB;
  constexpr int ARS = 256 / KT;   // row stride of the A_ROWS mapping
  static_assert(A_ROWS ? (256 % KT == 0 && BM == EA * ARS)
                       : A_MW ? (EA * ARW == KT)
                              : ((A_KCONTIG ? BM : KT) * TPRA == 256), "one pass over the A tile");
  static_assert(B_W ? (EB * ARW == KT) : (KT * TPRB == 256), "one pass over the B tile");
  const int am = A_ROWS ? tid / KT : A_MW ? tid % 64 : (A_KCONTIG ? tid / TPRA : (tid % TPRA) * EA);
  const int ak = A_ROWS ? tid % KT : A_MW ? tid / 64 : (A_KCONTIG ? (tid % TPRA) * EA : tid / TPRA);
  const int bk = B_W ? tid / 64 : tid / TPRB, bn = B_W ? tid % 64 : (tid % TPRB) * EB;
  // Per-thread operand pointers at k = koff of segment 0; a K tile advances
  // them by KT rows of k, a new segment moves them by sa_seg / sb_seg.
  const int kfirst = int(koff);
  const int M = run.mlim > 0 && run.mlim < d.M ? run.mlim : d.M;   // rows of A read (the rest read as zero)
  const int N = d.N;
  const int64_t sam = d.sam, sak = d.sak, sa_seg = d.sa_seg, ldb = d.ldb, sb_seg = d.sb_seg;
  const bool a_row_ok = A_KCONTIG ? (m0 + am < M) : true;
  const gbl<const T>* A0 = as_global(static_cast<const T*>(d.A)) + run.aptr;
  const gbl<const T>* pa = A0 + int64_t(m0 + am + run.amoff) * sam + int64_t(kfirst + ak + run.akoff) * sak;
  const gbl<const T>* cu = as_global(Cuser);
  const gbl<const T>* B0 = GATHER ? cu : as_global(static_cast<const T*>(d.B)) + run.bptr;
  const gbl<const T>* pb = GATHER ? cu : B0 + int64_t(kfirst + bk) * ldb + (n0 + bn);
  int kt_in_seg = 0;                          // K tile index within the current segment (next load)
  int seg_loaded = 0;
  // Gathered B: the rows of C for the next load's k rows, fetched one load
  // ahead so that the operand loads never wait on the index loads.  A
  // wave's k rows are uniform (B_W map), so the indices are scalar loads.
  static_assert(!GATHER || B_W, "gathered B uses the 64-wide row map");
  // Split modes: the 64 columns of a wave's B unit share chunk g = wave, so
  // its 8 k rows are again uniform.
  constexpr int NG = kSplit ? 8 : (B_W ? EB : 1);   // k rows of B per thread
  static_assert(!GATHER || !kSplit || UB == 1, "gathered split B: one unit per thread");
  int grow[NG];
  const cst<int32_t>* gidx_c = as_const(d.gidx);
  auto fetch_rows = [&](int kt) {
#pragma unroll
    for (int u = 0; u < NG; ++u) {
      const int krow = kSplit ? 8 * wave + u : bk + u * ARW;
      const int gk = __builtin_amdgcn_readfirstlane(kfirst + kt * KT + krow);
      grow[u] = gidx_c[gk < kend ? gk : kfirst];
    }
  };
  if constexpr (GATHER) {
    if (nsteps > 0) fetch_rows(0);
  }
  // An element outside its operand is read from gemm_zero: no branch, and
  // no select after the load that could make the MFMAs of the current K
  // tile wait for the loads in flight.
  const gbl<const T>* zero = as_global(reinterpret_cast<const T*>(gemm_zero));
  // Split modes: row (column) and chunk of each unit, and its operand offset
  // at k = koff of segment 0.
  int uam[UA], uag[UA], uac[UA], ubn[UB], ubg[UB], ubc[UB];   // uac, ubc: LDS chunk positions
  int64_t uao[UA], ubo[UB];
  if constexpr (kSplit) {
#pragma unroll
    for (int p = 0; p < UA; ++p) {
      const int c = tid + 256 * p;
      const bool in = c < BM * KC;
      uam[p] = !in ? 0 : A_KCONTIG ? c / KC : c % BM;
      uag[p] = !in ? 0 : A_KCONTIG ? c % KC : c / BM;
      uac[p] = split_chunk(uam[p], uag[p]);
      uao[p] = int64_t(m0 + uam[p] + run.amoff) * sam + int64_t(kfirst + 8 * uag[p] + run.akoff) * sak;
    }
#pragma unroll
    for (int p = 0; p < UB; ++p) {
      const int c = tid + 256 * p;
      const bool in = c < BN * KC;
      ubn[p] = in ? c % BN : 0;
      ubg[p] = in ? c / BN : 0;
      ubc[p] = split_chunk(ubn[p], ubg[p]);
      ubo[p] = int64_t(kfirst + 8 * ubg[p]) * ldb + (n0 + ubn[p]);
    }
  }
  int ld_step = 0;   // index of the next K tile to load; tiles past the last read as zero
  auto load = [&](int set) {
    const bool live = ld_step++ < nsteps;
    const int k0 = kfirst + kt_in_seg * KT;   // first k of this K tile
    const int64_t aoff = int64_t(seg_loaded) * sa_seg + int64_t(kt_in_seg) * KT * sak;
    if constexpr (kSplit) {
#pragma unroll
      for (int p = 0; p < UA; ++p) {
        const bool row_ok = live && tid + 256 * p < BM * KC && m0 + uam[p] < M;
        const int kc = k0 + 8 * uag[p];
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          const bool ok = row_ok && kc + e < kend;
          sa[set][p][e] = *(ok ? A0 + uao[p] + aoff + int64_t(e) * sak : zero);
        }
      }
      const int64_t boffk = int64_t(seg_loaded) * sb_seg + int64_t(kt_in_seg) * KT * ldb;
      if constexpr (GATHER) {
        int64_t roff[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          const int64_t r = int64_t(grow[e]) * ldcu + boff;
          const uint32_t lo = __builtin_amdgcn_readfirstlane(uint32_t(r));
          const uint32_t hi = __builtin_amdgcn_readfirstlane(uint32_t(uint64_t(r) >> 32));
          roff[e] = int64_t((uint64_t(hi) << 32) | lo);
        }
        const int gn = n0 + ubn[0], kc = k0 + 8 * ubg[0];
        const bool col_ok = live & (gn < N) & (boff + gn < blim);
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          const bool ok = col_ok & (kc + e < kend);
          sb[set][0][e] = *(ok ? cu + roff[e] + gn : zero);
        }
      } else {
#pragma unroll
        for (int p = 0; p < UB; ++p) {
          const bool col_ok = live && tid + 256 * p < BN * KC && n0 + ubn[p] < N;
          const int kc = k0 + 8 * ubg[p];
#pragma unroll
          for (int e = 0; e < 8; ++e) {
            const bool ok = col_ok && kc + e < kend;
            sb[set][p][e] = *(ok ? B0 + ubo[p] + boffk + int64_t(e) * ldb : zero);
          }
        }
      }
      if (++kt_in_seg == kpseg) {
        kt_in_seg = 0;
        ++seg_loaded;
      }
      if constexpr (GATHER) fetch_rows(kt_in_seg);
    } else {
#pragma unroll
    for (int u = 0; u < EA; ++u) {
      int64_t off;
      bool ok;
      if (A_ROWS) {
        ok = live && k0 + ak < kend && m0 + am + u * ARS < M;
        off = aoff + int64_t(u) * ARS * sam;
      } else if (A_KCONTIG) {
        ok = live && a_row_ok && k0 + ak + u < kend;
        off = aoff + int64_t(u) * sak;
      } else if (A_MW) {
        ok = live && k0 + ak + u * ARW < kend && m0 + am < M;
        off = aoff + int64_t(u) * ARW * sak;
      } else {
        ok = live && k0 + ak < kend && m0 + am + u < M;
        off = aoff + int64_t(u) * sam;
      }
      ra[set][u] = *(ok ? pa + off : zero);
    }
    const gbl<const T>* bplain = pb + int64_t(seg_loaded) * sb_seg + int64_t(kt_in_seg) * KT * ldb;
    // Gathered rows: offsets formed once per wave (readfirstlane is
    // convergent, so the compiler cannot sink them under the per-lane
    // bounds test and branch around the loads).
    int64_t roff[NG];
#pragma unroll
    for (int u = 0; u < NG; ++u) {
      const int64_t r = GATHER ? int64_t(grow[u]) * ldcu + boff : 0;
      const uint32_t lo = __builtin_amdgcn_readfirstlane(uint32_t(r));
      const uint32_t hi = __builtin_amdgcn_readfirstlane(uint32_t(uint64_t(r) >> 32));
      roff[u] = int64_t((uint64_t(hi) << 32) | lo);
    }
#pragma unroll
    for (int u = 0; u < EB; ++u) {
      const int kk = B_W ? bk + u * ARW : bk, gn = n0 + (B_W ? bn : bn + u);
      const bool ok = live & (k0 + kk < kend) & (gn < N) & (!GATHER | (boff + gn < blim));
      const gbl<const T>* p = GATHER ? cu + roff[B_W ? u : 0] + gn
                                     : bplain + (B_W ? int64_t(u) * ARW * ldb : int64_t(u));
      rb[set][u] = *(ok ? p : zero);
    }
    if (++kt_in_seg == kpseg) {
      kt_in_seg = 0;
      ++seg_loaded;
    }
    if constexpr (GATHER) fetch_rows(kt_in_seg);
    }
  };
  auto store = [&](int set, int buf) {
    if constexpr (kSplit) {
#pragma unroll
      for (int p = 0; p < UA; ++p) {
        if (tid + 256 * p >= BM * KC) continue;   // whole waves
        if constexpr (MODE == kModeBF16x6)
          split8x3(sa[set][p], sm.A[buf][0][uam[p]][uac[p]], sm.A[buf][1][uam[p]][uac[p]],
                   sm.A[buf][2][uam[p]][uac[p]]);
        else
          split8(sa[set][p], sm.A[buf][0][uam[p]][uac[p]], sm.A[buf][1][uam[p]][uac[p]]);
      }
#pragma unroll
      for (int p = 0; p < UB; ++p) {
        if (tid + 256 * p >= BN * KC) continue;
        if constexpr (MODE == kModeBF16x6)
          split8x3(sb[set][p], sm.B[buf][0][ubn[p]][ubc[p]], sm.B[buf][1][ubn[p]][ubc[p]],
                   sm.B[buf][2][ubn[p]][ubc[p]]);
        else
          split8(sb[set][p], sm.B[buf][0][ubn[p]][ubc[p]], sm.B[buf][1][ubn[p]][ubc[p]]);
      }
    } else {
    auto& Aw = sm.A[buf];
    auto& Bw = sm.B[buf];
#pragma unroll
    for (int u = 0; u < EA; ++u) {
      const T v = ra[set][u];
      if (A_ROWS) Aw[ak][am + u * ARS] = v;
      else if (A_KCONTIG) Aw[ak + u][am] = v;
      else if (A_MW) Aw[ak + u * ARW][am] = v;
      else Aw[ak][am + u] = v;
    }
#pragma unroll
    for (int u = 0; u < EB; ++u) {
      if (B_W) Bw[bk + u * ARW][bn] = rb[set][u];
      else Bw[bk][bn + u] = rb[set][u];
    }
    }
  };
  auto compute = [&](int cur) {
    if constexpr (kSplit) {
      // one 16-byte LDS read per plane and fragment; planes 0, 1 (, 2) are
      // hi, (mid,) lo
      constexpr int NP = mode_planes(MODE);
      const int fr = lane & 15, fg = lane >> 4;
      bf16x8 a[NP][TM], b[NP][TN];
      const int fc = split_chunk(fr, fg);   // rows wm + 16 i + fr: wm, 16 i are multiples of 16
      for (int j = 0; j < TN; ++j)
        for (int p = 0; p < NP; ++p) b[p][j] = sm.B[cur][p][wn + j * 16 + fr][fc];
      for (int i = 0; i < TM; ++i)
        for (int p = 0; p < NP; ++p) a[p][i] = sm.A[cur][p][wm + i * 16 + fr][fc];
      for (int i = 0; i < TM; ++i)
        for (int j = 0; j < TN; ++j) {   // smallest terms first
          if constexpr (MODE == kModeBF16x6) {
            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[1][i], b[1][j], acc[i][j], 0, 0, 0);
            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[2][i], b[0][j], acc[i][j], 0, 0, 0);
            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[0][i], b[2][j], acc[i][j], 0, 0, 0);
            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[1][i], b[0][j], acc[i][j], 0, 0, 0);
            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[0][i], b[1][j], acc[i][j], 0, 0, 0);
          } else {
            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[1][i], b[0][j], acc[i][j], 0, 0, 0);
            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[0][i], b[1][j], acc[i][j], 0, 0, 0);
          }
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[0][i], b[0][j], acc[i][j], 0, 0, 0);
        }
    } else {
      auto& As = sm.A[cur];
      auto& Bs = sm.B[cur];
#pragma unroll
      for (int kk = 0; kk < KT; kk += 4) {
        const int kr = kk + (lane >> 4);
        T a[TM], b[TN];
        for (int i = 0; i < TM; ++i) a[i] = As[kr][wm + i * 16 + (lane & 15)];
        for (int j = 0; j < TN; ++j) b[j] = Bs[kr][wn + j * 16 + (lane & 15)];
        for (int i = 0; i < TM; ++i)
          for (int j = 0; j < TN; ++j) acc[i][j] = mfma4(a[i], b[j], acc[i][j]);
      }
    }
  };
  auto flush = [&]() {
    if constexpr (kFlush) {
      if (++ktile == FLUSH) {
        ktile = 0;
        for (int i = 0; i < TM; ++i)
          for (int j = 0; j < TN; ++j) {
            for (int r = 0; r < 4; ++r) acc64[i][j][r] += double(acc[i][j][r]);
            acc[i][j] = Acc{};
          }
      }
    }
  };

  // DEPTH = 2: tile s is computed from LDS buffer s & 1 while tile s + 1
  // waits in one register set and tiles s + 2, s + 3 are loaded; the loop
  // runs two K tiles per iteration so that register sets and buffers are
  // fixed.  DEPTH = 1, NB = 2: loads one tile ahead, one barrier per tile.
  // NB = 1: one buffer, loads one tile ahead, two barriers per tile.
  // Stores and loads past the last tile move zeros and keep the loops free
  // of branches.
  if (nsteps > 0) {
    if constexpr (DEPTH == 2) {
      load(0);
      store(0, 0);
      __syncthreads();
      load(1);
      load(0);
      int step = 0;
      for (; step + 2 <= nsteps; step += 2) {
        compute(0);
        store(1, 1);   // buffer 1's last readers passed the previous barrier
        load(1);
        __syncthreads();
        flush();
        compute(1);
        store(0, 0);
        load(0);
        __syncthreads();
        flush();
      }
      if (step < nsteps) {
        compute(0);
        flush();
      }
    } else if constexpr (NB == 2) {
      load(0);
      store(0, 0);
      __syncthreads();
      for (int step = 0; step + 1 < nsteps; ++step) {
        const int cur = step & 1;
        load(0);
        compute(cur);
        store(0, cur ^ 1);   // the other buffer's last readers passed the previous barrier
        __syncthreads();
        flush();
      }
      compute((nsteps - 1) & 1);
      flush();
    } else {
      load(0);
      for (int step = 0; step + 1 < nsteps; ++step) {
        store(0, 0);
        __syncthreads();
        load(0);
        compute(0);
        __syncthreads();
        flush();
      }
      store(0, 0);
      __syncthreads();
      compute(0);
      flush();
    }
  }
  if constexpr (kFlush)
    for (int i = 0; i < TM; ++i)
      for (int j = 0; j < TN; ++j)
        for (int r = 0; r < 4; ++r) acc64[i][j][r] += double(acc[i][j][r]);
  gbl<OutT>* Cout = as_global(static_cast<OutT*>(d.C)) + run.coff;
  const int64_t ldcn = d.ldcn ? d.ldcn : 1;
  const int mend = run.mlim > 0 && run.mlim < d.M ? run.mlim : d.M;
  for (int i = 0; i < TM; ++i)
    for (int j = 0; j < TN; ++j) {
      const int col = n0 + wn + j * 16 + (lane & 15);
      if (col >= d.N || col < run.nlo || (run.nhi > 0 && col >= run.nhi)) continue;
      for (int r = 0; r < 4; ++r) {
        const int row = m0 + wm + i * 16 + acc_row<Acc>(lane >> 4, r);
        if (row >= mend) continue;
        gbl<OutT>* c = Cout + int64_t(row) * d.ldc + int64_t(col) * ldcn;
        OutT v;
        if constexpr (kFlush) v = OutT(acc64[i][j][r]);
        else v = OutT(acc[i][j][r]);
        if (run.accumulate) *c = *c + v;
        else store_stream(c, v);
      }
    }
  __syncthreads();   // LDS is reused by the caller's next tile
}

template <int MODE, bool A_KCONTIG, bool GATHER, class OutT, class S, int NB, int DEPTH>
__device__ __forceinline__ void gemm_grouped(const GemmDesc* __restrict__ descs, const GemmTile* __restrict__ tiles,
                                             const typename ModeT<MODE>::T* __restrict__ Cuser, int64_t ldcu,
                                             const GemmRun& run) {
  __shared__ GemmSmem<MODE, S, NB> sm;
  // XCD-aware order: the grid is a multiple of 8 and hardware block b runs on
  // XCD b % 8, so XCD x walks the contiguous tile range [x*per, (x+1)*per).
  // Tiles that share an operand panel are adjacent in the list and hence
  // share one L2.
  const int per = int(gridDim.x / 8);
  const int logical = int(blockIdx.x % 8) * per + int(blockIdx.x / 8);
  if (logical >= run.ntiles) return;
  const GemmTile tl = tiles[run.tile0 + logical];
  gemm_tile<MODE, A_KCONTIG, GATHER, OutT, S, NB, DEPTH>(descs[tl.prob], tl.mt, tl.nt, Cuser, ldcu, run, sm);
}

// One kernel per contraction, so that profiles name the step:
//   half_kernel   H = O C (Eq. 15a), per j batch and for all columns (HT)
//   omega_kernel  Omega = H^T C (Eq. 15b)
//   l2p_kernel    K partials from the carried columns (Eq. 18)
//   l2pt_kernel   K partials from the mirrored columns (Eq. 18, symmetric schedule)
//   l2p_wide_kernel, l2pt_wide_kernel  the same with a whole leaf per tile
//   omega_ht_kernel, l2p_ht_kernel, l2p_ht_wide_kernel  Omega and L2P with
//                 the batch's H read out of HT (symmetric schedule)
#define OCCK_GEMM_KERNEL(NAME, AK, GA, OUT, SHAPE, NB, DEPTH)                                                  \
  template <int MODE>                                                                                          \
  __global__ __launch_bounds__(256) void NAME(const GemmDesc* __restrict__ descs,                              \
                                              const GemmTile* __restrict__ tiles,                              \
                                              const typename ModeT<MODE>::T* __restrict__ Cuser, int64_t ldcu, \
                                              GemmRun run) {                                                   \
    gemm_grouped<MODE, AK, GA, OUT, SHAPE, NB, DEPTH>(descs, tiles, Cuser, ldcu, run);                           \
  }
// Loads two K tiles ahead only in l2p (a long K loop over the (q, j) rows of
// Mloc); half and omega contract over the n_B functions of a leaf (a few K
// tiles), in l2pt the deeper loads cost more in L2 misses (the tiles of one
// leaf drift apart) than they gain in latency, and the whole-leaf tiles
// would drop to 2 waves per SIMD.
OCCK_GEMM_KERNEL(half_kernel, true, true, typename ModeT<MODE>::T, GemmRows48, (MODE == kModeBF16x6 ? 1 : 2), 1)
OCCK_GEMM_KERNEL(omega_kernel, false, true, typename ModeT<MODE>::T, GemmSquare, (MODE == kModeBF16x6 ? 1 : 2), 1)
OCCK_GEMM_KERNEL(l2p_kernel, true, false, double, GemmRows48, 2, 2)
OCCK_GEMM_KERNEL(l2pt_kernel, true, false, double, GemmCols48, 2, 1)
OCCK_GEMM_KERNEL(l2pt_wide_kernel, true, false, double, GemmCols144, 2, 1)
OCCK_GEMM_KERNEL(l2p_wide_kernel, true, false, double, GemmRows144, 2, 1)
// The symmetric schedule reads the half transform of a j batch out of HT
// (formed once per call for every column) instead of forming it per batch:
// A is HT^B_q[i][t] (t contiguous), Omega per (leaf, q) with rows j, and the
// direct L2P over K segments q with k = j.
OCCK_GEMM_KERNEL(omega_ht_kernel, true, true, typename ModeT<MODE>::T, GemmSquare, (MODE == kModeBF16x6 ? 1 : 2), 1)
OCCK_GEMM_KERNEL(l2p_ht_kernel, false, false, double, GemmRows48, 2, 2)
OCCK_GEMM_KERNEL(l2p_ht_wide_kernel, false, false, double, GemmRows144, 2, 1)
#undef OCCK_GEMM_KERNEL

// --------------------------------------------------------------------------
// translation: out[t] = sum_{e in CSR(t)} T[op_e] * data[src_e]   (overwrite)
// Each box is Q rows x ncol columns.  Block = 4 waves x 64 columns; each wave
// holds MT 16-row tiles x 4 column tiles of accumulators.  Blocks are
// renumbered so that each XCD walks contiguous (column tile, target) ranges:
// neighbouring targets then share their sources in that XCD's L2.
// T = double: FP64 MFMA; T = float: FP32 MFMA.
// --------------------------------------------------------------------------
// src_rank (may be null): per CSR entry the rank p kept in that translation
// (components l, l' <= p, i.e. the leading (p+1)^2 rows and columns).
// USE_LDS: op_lds is a block-shared staging area of at least MT*KS*64
// elements; the 256 threads copy each source's operator into it once and the
// four waves read their A fragments from LDS (one global read of the
// operator per block instead of one per wave).  The block then must call
// this routine with all its threads.
// perm (may be null; not with src_rank): the operators hold the components
// in the order perm lists them, grouped by reflection class (pcls: class of
// each position, non-decreasing).  Source rows are read and target rows
// written at perm[position], and an operator block (16 rows x one k step of
// 4) whose row and column classes do not meet is a structural zero: its
// products are skipped.  perm_lds holds perm for the block.
template <class T, int MT, bool USE_LDS, bool PERM = false>
__device__ void translate_tile(T* __restrict__ data, int64_t box_stride, const ColMap& cm, int Q, int KS,
                               const int32_t* __restrict__ tgt_box, const int32_t* __restrict__ src_ptr,
                               const int32_t* __restrict__ src_box, const int32_t* __restrict__ src_op,
                               const T* __restrict__ ops, int t, int64_t ct, const int8_t* __restrict__ src_rank,
                               T* __restrict__ op_lds, const int32_t* __restrict__ perm = nullptr,
                               const int8_t* __restrict__ pcls = nullptr, int32_t* __restrict__ perm_lds = nullptr) {
  using Acc = typename std::conditional<std::is_same<T, double>::value, d4, f4>::type;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t ncol = cm.ncol;
  const int64_t vbase = ct * 256 + wave * 64;
  int64_t cols[4];
  bool ok[4];
  for (int j = 0; j < 4; ++j) {
    const int64_t v = vbase + j * 16 + (lane & 15);
    ok[j] = v < cm.nvalid;
    cols[j] = ok[j] ? carried_col(cm, v) : 0;
  }
  Acc acc[MT][4];
  for (int i = 0; i < MT; ++i)
    for (int j = 0; j < 4; ++j) acc[i][j] = Acc{};
  const int64_t opsz = int64_t(MT) * KS * 64;
  const cst<int32_t>* sbox = as_const(src_box);
  const cst<int32_t>* sop = as_const(src_op);
  const int e0 = as_const(src_ptr)[t], e1 = as_const(src_ptr)[t + 1];
  constexpr bool permuted = PERM;
  if constexpr (PERM) {
    for (int q = threadIdx.x; q < Q; q += 256) perm_lds[q] = perm[q];
    __syncthreads();
  }
  // block (row tile i, k step ks) holds nonzero entries (classes of its
  // rows and columns meet): bit i*KS + ks of a block-uniform mask (MT * KS
  // <= 6 * 24 = 144 bits), formed once per block
  uint64_t lmask[3] = {~0ull, ~0ull, ~0ull};
  if constexpr (PERM) {
    static_assert(MT * 4 * MT <= 192, "live mask size");
    lmask[0] = lmask[1] = lmask[2] = 0;
    const cst<int8_t>* c = as_const(pcls);
    for (int i = 0; i < MT; ++i)
      for (int ks = 0; ks < KS; ++ks) {
        const int r0 = i * 16, r1 = min(r0 + 15, Q - 1), k0 = ks * 4, k1 = min(k0 + 3, Q - 1);
        if (r0 < Q && c[r0] <= c[k1] && c[k0] <= c[r1]) {
          const int bit = i * KS + ks;
          lmask[bit >> 6] |= 1ull << (bit & 63);
        }
      }
  }
  auto live = [&](int i, int ks) {
    if constexpr (!PERM) return true;
    const int bit = i * KS + ks;
    return ((lmask[bit >> 6] >> (bit & 63)) & 1ull) != 0;
  };
  for (int e = e0; e < e1; ++e) {
    const gbl<const T>* X = as_global(static_cast<const T*>(data)) + int64_t(sbox[e]) * box_stride;
    const gbl<const T>* Tm = as_global(ops) + int64_t(sop[e]) * opsz;
    int nq = Q, kse = KS;
    if (src_rank) {
      const int p = as_global(src_rank)[e];
      nq = (p + 1) * (p + 1);
      kse = (nq + 3) / 4;
    }
    const int nfi = (nq + 15) / 16;   // row tiles in use (<= MT)
    if constexpr (USE_LDS) {
      __syncthreads();   // every wave is done with the previous operator
      for (int idx = threadIdx.x; idx < MT * KS * 64; idx += 256) {
        const int frag = idx >> 6, i = frag / KS, ks = frag - i * KS;
        if (i < nfi && ks < kse && live(i, ks)) op_lds[idx] = Tm[idx];
      }
      __syncthreads();
    }
    // Branch-free operand loads: every address is in bounds (rows clamped to
    // Q - 1, invalid columns read column 0) and invalid values are replaced
    // by zero afterwards.  The next k step's B fragments are in flight
    // during this step's MFMAs.
    T bn[4];   // raw values of the next k step (masked when used)
    auto loadb = [&](int ks, T (&b)[4]) {
      const int row = ks * 4 + (lane >> 4);
      const int rc0 = row < Q ? row : Q - 1;
      const int rc = permuted ? perm_lds[rc0] : rc0;
      for (int j = 0; j < 4; ++j) b[j] = X[int64_t(rc) * ncol + cols[j]];
    };
    if (kse > 0) loadb(0, bn);
    for (int ks = 0; ks < kse; ++ks) {
      const bool row_ok = ks * 4 + (lane >> 4) < Q;
      T b[4];
      for (int j = 0; j < 4; ++j) b[j] = (row_ok && ok[j]) ? bn[j] : T(0);
      if (ks + 1 < kse) loadb(ks + 1, bn);
      T a[MT];
#pragma unroll
      for (int i = 0; i < MT; ++i) {
        const int64_t fi = (int64_t(i) * KS + ks) * 64 + lane;
        if constexpr (USE_LDS)
          a[i] = op_lds[fi];
        else
          a[i] = T(Tm[fi]);
      }
      if (nq < Q) {   // truncated rank: entries with l or l' above p are zero
        const int row = ks * 4 + (lane >> 4);
#pragma unroll
        for (int i = 0; i < MT; ++i)
          if (i * 16 + (lane & 15) >= nq || row >= nq) a[i] = T(0);
      }
#pragma unroll
      for (int i = 0; i < MT; ++i)   // row tiles beyond the rank, and structural-zero blocks, are skipped
        if (i < nfi && live(i, ks))
          for (int j = 0; j < 4; ++j) acc[i][j] = mfma4(a[i], b[j], acc[i][j]);
    }
  }
  gbl<T>* Y = as_global(data) + int64_t(as_const(tgt_box)[t]) * box_stride;
  for (int i = 0; i < MT; ++i)
    for (int j = 0; j < 4; ++j) {
      if (!ok[j]) continue;
      for (int r = 0; r < 4; ++r) {
        const int row = i * 16 + acc_row<Acc>(lane >> 4, r);
        if (row < Q) store_stream(Y + int64_t(permuted ? perm_lds[row] : row) * ncol + cols[j], T(acc[i][j][r]));
      }
    }
}

template <class T, int MT>
__global__ __launch_bounds__(256) void translate_kernel(T* __restrict__ data, int64_t box_stride, ColMap cm,
                                                        int Q, int KS, const int32_t* __restrict__ tgt_box,
                                                        const int32_t* __restrict__ src_ptr,
                                                        const int32_t* __restrict__ src_box,
                                                        const int32_t* __restrict__ src_op,
                                                        const T* __restrict__ ops, int ntgt, int64_t nblocks,
                                                        const int8_t* __restrict__ src_rank) {
  __shared__ T op_lds[MT * 4 * MT * 64];   // KS <= 4 MT
  const int64_t per = (int64_t(gridDim.x) + 7) / 8;
  const int64_t logical = int64_t(blockIdx.x % 8) * per + blockIdx.x / 8;
  if (logical >= nblocks) return;   // block-uniform
  translate_tile<T, MT, true>(data, box_stride, cm, Q, KS, tgt_box, src_ptr, src_box, src_op, ops,
                              int(logical % ntgt), logical / ntgt, src_rank, op_lds);
}

// The same with the operators in class order (perm, pcls): structural-zero
// blocks skipped (fixed ranks only).
template <class T, int MT>
__global__ __launch_bounds__(256) void translate_perm_kernel(T* __restrict__ data, int64_t box_stride, ColMap cm,
                                                             int Q, int KS, const int32_t* __restrict__ tgt_box,
                                                             const int32_t* __restrict__ src_ptr,
                                                             const int32_t* __restrict__ src_box,
                                                             const int32_t* __restrict__ src_op,
                                                             const T* __restrict__ ops, int ntgt, int64_t nblocks,
                                                             const int32_t* __restrict__ perm,
                                                             const int8_t* __restrict__ pcls) {
  __shared__ T op_lds[MT * 4 * MT * 64];   // KS <= 4 MT
  __shared__ int32_t perm_lds[MT * 16];
  const int64_t per = (int64_t(gridDim.x) + 7) / 8;
  const int64_t logical = int64_t(blockIdx.x % 8) * per + blockIdx.x / 8;
  if (logical >= nblocks) return;   // block-uniform
  translate_tile<T, MT, true, true>(data, box_stride, cm, Q, KS, tgt_box, src_ptr, src_box, src_op, ops,
                                    int(logical % ntgt), logical / ntgt, nullptr, op_lds, perm, pcls, perm_lds);
}

// --------------------------------------------------------------------------
// Structural zeros of axis-aligned translations.  A box centre takes the
// root's midpoint in every unsplit dimension, so on a tree split along x
// only, every translation displacement lies on the x axis, and on a tree
// not split along z, in the xy plane.  Such a displacement is unchanged by
// the reflection z -> -z, under which a real component (l, m, Re|Im) picks
// up (-1)^(l+m), and the x-axis one also by y -> -y, which flips the sign of
// the Im components only.  The translation operators (Eqs. 11-13) commute
// with these reflections, so T[q][q'] vanishes unless q and q' have the same
// signs; the recurrences of the harmonics produce those zeros exactly (a
// zero y or z propagates as an exact zero), so skipping them changes no
// result.  SYM 0: dense; 1: displacements on the x axis (four classes,
// 25 of the 81 entries at L = 2); 2: displacements in the xy plane (two
// classes, 45 of 81).
// --------------------------------------------------------------------------
__host__ __device__ constexpr int real_class(int q, int sym) {
  int l = 0;
  while ((l + 1) * (l + 1) <= q) ++l;
  const int k = q - l * l;
  const int m = (k + 1) / 2;
  const int im = (k != 0 && (k & 1) == 0) ? 1 : 0;
  return sym == 1 ? 2 * im + ((l + m) & 1) : sym == 2 ? ((l + m) & 1) : 0;
}
__host__ __device__ constexpr bool op_entry_live(int i, int k, int sym) {
  return real_class(i, sym) == real_class(k, sym);
}

// --------------------------------------------------------------------------
// Exact-size translations for Q <= 9 (L <= 2) on the vector ALU.  On gfx950
// the FP64 MFMA peak equals the FP64 vector FMA peak, and a 9x9 operator
// padded to 16x12 MFMA tiles issues 2.4x the useful products, so small
// translations run as plain FMAs: each thread owns NC columns (lane-
// consecutive, 512-byte wave loads per component row), the operator entries
// are wave-uniform loads from the fragment-ordered operator (scalar cache),
// and every product is one FMA into an FP64 (or FP32) accumulator.  Per
// source: Q loads and Q*Q FMAs per column.  Same CSR passes, same XCD-aware
// block order as translate_kernel; block covers 256*NC columns of one target.
// --------------------------------------------------------------------------
// PIPE: the next source's column values are loaded while the current one's
// products are formed (two register sets); without it, one source at a time.
template <class T, int Q, int NC, int SYM, bool PIPE = true>
__device__ void translate_vec_tile(T* __restrict__ data, int64_t box_stride, const ColMap& cm, int KS,
                                   const int32_t* __restrict__ tgt_box, const int32_t* __restrict__ src_ptr,
                                   const int32_t* __restrict__ src_box, const int32_t* __restrict__ src_op,
                                   const double* __restrict__ ops, int t, int64_t ct) {
  static_assert(Q <= 16, "one operator row tile");
  const int64_t v0 = ct * (256 * NC) + threadIdx.x;
  const int64_t ncol = cm.ncol;
  bool ok[NC];
  int64_t col[NC];
  for (int c = 0; c < NC; ++c) {
    ok[c] = v0 + c * 256 < cm.nvalid;
    col[c] = ok[c] ? carried_col(cm, v0 + c * 256) : 0;
  }
  // FP64 operators and accumulators in every mode: a target sums up to a few
  // hundred terms per component (3-D interaction lists), which FP32 sums
  // would round to ~1e-6; the products cost the same on the vector ALU
  double acc[NC][Q];
  for (int c = 0; c < NC; ++c)
    for (int i = 0; i < Q; ++i) acc[c][i] = 0.0;
  const int64_t opsz = int64_t(KS) * 64;
  const cst<int32_t>* sbox = as_const(src_box);
  const cst<int32_t>* sop = as_const(src_op);
  const int e0 = as_const(src_ptr)[t], e1 = as_const(src_ptr)[t + 1];
  // Raw column values of the next source are in flight while the current
  // source's products are formed (two register sets, used alternately).
  // Addresses are always in bounds (invalid columns read column 0); the
  // values of invalid columns are never stored.
  const gbl<const T>* base = as_global(static_cast<const T*>(data));
  T xa[NC][Q], xb[NC][Q];
  auto fetch = [&](T (&x)[NC][Q], int e) {
    const gbl<const T>* X = base + int64_t(sbox[e]) * box_stride;
    for (int c = 0; c < NC; ++c)
      for (int k = 0; k < Q; ++k) x[c][k] = X[int64_t(k) * ncol + col[c]];
  };
  auto apply = [&](const T (&x)[NC][Q], int e) {
    const cst<double>* A = as_const(ops) + int64_t(sop[e]) * opsz;
    double xd[NC][Q];
    for (int c = 0; c < NC; ++c)
      for (int k = 0; k < Q; ++k) xd[c][k] = double(x[c][k]);
#pragma unroll
    for (int i = 0; i < Q; ++i)
#pragma unroll
      for (int k = 0; k < Q; ++k) {
        if (!op_entry_live(i, k, SYM)) continue;   // a structural zero
        const double a = A[(k >> 2) * 64 + i + 16 * (k & 3)];   // T[i][k]
        for (int c = 0; c < NC; ++c) acc[c][i] = fma(a, xd[c][k], acc[c][i]);
      }
  };
  if constexpr (PIPE) {
    if (e0 < e1) fetch(xa, e0);
    for (int e = e0; e < e1; e += 2) {
      if (e + 1 < e1) fetch(xb, e + 1);
      apply(xa, e);
      if (e + 1 >= e1) break;
      if (e + 2 < e1) fetch(xa, e + 2);
      apply(xb, e + 1);
    }
  } else {
    for (int e = e0; e < e1; ++e) {
      fetch(xa, e);
      apply(xa, e);
    }
  }
  gbl<T>* Y = as_global(data) + int64_t(as_const(tgt_box)[t]) * box_stride;
  for (int c = 0; c < NC; ++c)
    if (ok[c])
      for (int i = 0; i < Q; ++i) store_stream(Y + int64_t(i) * ncol + col[c], T(acc[c][i]));
}

template <class T, int Q, int NC, int SYM>
__global__ __launch_bounds__(256) void translate_vec_kernel(T* __restrict__ data, int64_t box_stride, ColMap cm,
                                                            int KS, const int32_t* __restrict__ tgt_box,
                                                            const int32_t* __restrict__ src_ptr,
                                                            const int32_t* __restrict__ src_box,
                                                            const int32_t* __restrict__ src_op,
                                                            const double* __restrict__ ops, int ntgt, int64_t nblocks) {
  const int64_t per = (int64_t(gridDim.x) + 7) / 8;
  const int64_t logical = int64_t(blockIdx.x % 8) * per + blockIdx.x / 8;
  if (logical >= nblocks) return;
  translate_vec_tile<T, Q, NC, SYM>(data, box_stride, cm, KS, tgt_box, src_ptr, src_box, src_op, ops,
                               int(logical % ntgt), logical / ntgt);
}

// --------------------------------------------------------------------------
// upward pass as a walk (M2M, Eqs. 11 and 17a): one block per (subtree below a box of
// the walk's root level, 256 carried columns), one column per thread.  The
// block runs the subtree's post-order program: UP_LEAF adds T_op M(leaf)
// into the accumulator of the leaf's parent level; UP_CLOSE stores a
// finished box's M and adds T_op M(box) into its parent's accumulator (op <
// 0: the subtree root).  Internal boxes are written once and never read
// back, and every accumulator takes the same FMA sequence as the
// level-by-level passes.  Accumulators are indexed by level relative to the
// root level (NLV levels in registers); the next leaf's column values are in
// flight while the current program step runs.
// --------------------------------------------------------------------------
struct WalkStep {   // one step of an upward or downward walk program
  int32_t kind;    // UP_LEAF, UP_CLOSE (upward); DN_BEGIN, DN_SRC, DN_STORE (downward)
  int32_t level;   // accumulator: tree level minus the walk's root level
  int32_t box;     // box slot read (UP_LEAF, DN_SRC) or written (UP_CLOSE, DN_STORE)
  int32_t op;      // operator of the step's term (-1: none)
};
enum { UP_LEAF = 0, UP_CLOSE = 1 };
constexpr int kUpWalkLevels = 6;   // accumulator levels (below the walk's root level) held in registers

// load_shift: box rows added to every leaf read (a second leaf Omega region,
// so that the next j batch's Omega can be formed while this walk runs).
template <class T, int Q, int NLV, int SYM>
__global__ __launch_bounds__(256) void up_walk_kernel(T* __restrict__ data, int64_t box_stride, ColMap cm, int KS,
                                                      const int32_t* __restrict__ prog_ptr,
                                                      const WalkStep* __restrict__ prog, const T* __restrict__ ops,
                                                      int nroots, int64_t nblocks, int64_t load_shift) {
  const int64_t per = (int64_t(gridDim.x) + 7) / 8;
  const int64_t logical = int64_t(blockIdx.x % 8) * per + blockIdx.x / 8;
  if (logical >= nblocks) return;
  const int root = int(logical % nroots);
  const int64_t ct = logical / nroots;
  const int64_t v = ct * 256 + threadIdx.x;
  const bool ok = v < cm.nvalid;
  const int64_t col = ok ? carried_col(cm, v) : 0;   // invalid columns read column 0, store nothing
  const int64_t ncol = cm.ncol;
  const int64_t opsz = int64_t(KS) * 64;
  const gbl<const T>* base = as_global(static_cast<const T*>(data));
  const cst<WalkStep>* pg = as_const(prog);
  const int p0 = as_const(prog_ptr)[root], p1 = as_const(prog_ptr)[root + 1];
  // the walks run on chain-like trees, whose interaction lists are short:
  // the accumulators take few terms, and the mode's precision is kept
  T acc[NLV][Q];
#pragma unroll
  for (int l = 0; l < NLV; ++l)
#pragma unroll
    for (int i = 0; i < Q; ++i) acc[l][i] = T(0);
  // y += T_op x, in the order of the level-by-level kernel
  auto apply = [&](T (&y)[Q], const T (&x)[Q], int op) {
    const cst<T>* A = as_const(ops) + int64_t(op) * opsz;
#pragma unroll
    for (int i = 0; i < Q; ++i)
#pragma unroll
      for (int k = 0; k < Q; ++k)
        if (op_entry_live(i, k, SYM)) y[i] = fma(A[(k >> 2) * 64 + i + 16 * (k & 3)], x[k], y[i]);
  };
  auto next_leaf = [&](int s) {
    while (s < p1 && pg[s].kind != UP_LEAF) ++s;
    return s;
  };
  T xn[Q];
  auto fetch = [&](int s) {   // column values of the leaf of step s (s < p1)
    const gbl<const T>* X = base + (int64_t(pg[s].box) + load_shift) * box_stride;
    for (int k = 0; k < Q; ++k) xn[k] = X[int64_t(k) * ncol + col];
  };
  int nl = next_leaf(p0);
  if (nl < p1) fetch(nl);
  for (int s = p0; s < p1; ++s) {
    const WalkStep in = load_const(prog + s);
    if (in.kind == UP_LEAF) {
      T x[Q];
      for (int k = 0; k < Q; ++k) x[k] = xn[k];
      nl = next_leaf(s + 1);
      if (nl < p1) fetch(nl);
#pragma unroll
      for (int l = 0; l < NLV; ++l)
        if (l == in.level) apply(acc[l], x, in.op);
    } else {
      gbl<T>* Y = as_global(data) + int64_t(in.box) * box_stride;
#pragma unroll
      for (int l = 0; l < NLV; ++l)
        if (l == in.level) {
          if (ok)
            for (int i = 0; i < Q; ++i) store_stream(Y + int64_t(i) * ncol + col, acc[l][i]);
          if (l > 0 && in.op >= 0) apply(acc[l > 0 ? l - 1 : 0], acc[l], in.op);
          for (int i = 0; i < Q; ++i) acc[l][i] = T(0);
        }
    }
  }
}

// --------------------------------------------------------------------------
// downward pass as a walk (L2L and M2L, Eqs. 12, 13 and 17b,c): one block per (subtree
// below a box of the walk's root level, 256 carried columns), one column per
// thread, in pre-order.  DN_BEGIN opens a box at a level: its accumulator starts at
// zero and takes T_op L(parent) from the parent level's accumulator (op < 0:
// a subtree root, which has no parent term); DN_SRC adds T_op M(box) of an
// interaction-list source; DN_STORE writes a leaf's local expansion.  The
// local expansions above the leaves stay in registers and are never
// written; every accumulator takes the terms in the order of the
// level-by-level passes (parent first, then the interaction list).
// --------------------------------------------------------------------------
enum { DN_BEGIN = 0, DN_SRC = 1, DN_STORE = 2 };
constexpr int kDownWalkLevels = 2;   // accumulator levels (root level..D) held in registers

// store_shift: box rows added to every stored leaf; src_shift: box rows
// added to every source in [src_lo, src_hi) (second leaf Mloc and leaf
// Omega regions, so that two j batches can be in flight).
template <class T, int Q, int NLV, int SYM>
__global__ __launch_bounds__(256) void down_walk_kernel(T* __restrict__ data, int64_t box_stride, ColMap cm, int KS,
                                                        const int32_t* __restrict__ prog_ptr,
                                                        const WalkStep* __restrict__ prog, const T* __restrict__ ops,
                                                        int nroots, int64_t nblocks, int64_t store_shift,
                                                        int64_t src_shift, int32_t src_lo, int32_t src_hi) {
  const int64_t per = (int64_t(gridDim.x) + 7) / 8;
  const int64_t logical = int64_t(blockIdx.x % 8) * per + blockIdx.x / 8;
  if (logical >= nblocks) return;
  const int root = int(logical % nroots);
  const int64_t ct = logical / nroots;
  const int64_t v = ct * 256 + threadIdx.x;
  const bool ok = v < cm.nvalid;
  const int64_t col = ok ? carried_col(cm, v) : 0;   // invalid columns read column 0, store nothing
  const int64_t ncol = cm.ncol;
  const int64_t opsz = int64_t(KS) * 64;
  const gbl<const T>* base = as_global(static_cast<const T*>(data));
  const cst<WalkStep>* pg = as_const(prog);
  const int p0 = as_const(prog_ptr)[root], p1 = as_const(prog_ptr)[root + 1];
  // the walks run on chain-like trees, whose interaction lists are short:
  // the accumulators take few terms, and the mode's precision is kept
  T acc[NLV][Q];
#pragma unroll
  for (int l = 0; l < NLV; ++l)
#pragma unroll
    for (int i = 0; i < Q; ++i) acc[l][i] = T(0);
  auto apply = [&](T (&y)[Q], const T (&x)[Q], int op) {   // y += T_op x, as the level-by-level kernel
    const cst<T>* A = as_const(ops) + int64_t(op) * opsz;
#pragma unroll
    for (int i = 0; i < Q; ++i)
#pragma unroll
      for (int k = 0; k < Q; ++k)
        if (op_entry_live(i, k, SYM)) y[i] = fma(A[(k >> 2) * 64 + i + 16 * (k & 3)], x[k], y[i]);
  };
  auto next_src = [&](int s) {
    while (s < p1 && pg[s].kind != DN_SRC) ++s;
    return s;
  };
  T xn[Q];
  auto fetch = [&](int s) {   // column values of the source of step s (s < p1)
    const int32_t box = pg[s].box;
    const gbl<const T>* X = base + (int64_t(box) + (box >= src_lo && box < src_hi ? src_shift : 0)) * box_stride;
    for (int k = 0; k < Q; ++k) xn[k] = X[int64_t(k) * ncol + col];
  };
  int ns = next_src(p0);
  if (ns < p1) fetch(ns);
  for (int s = p0; s < p1; ++s) {
    const WalkStep in = load_const(prog + s);
    if (in.kind == DN_SRC) {
      T x[Q];
      for (int k = 0; k < Q; ++k) x[k] = xn[k];
      ns = next_src(s + 1);
      if (ns < p1) fetch(ns);
#pragma unroll
      for (int l = 0; l < NLV; ++l)
        if (l == in.level) apply(acc[l], x, in.op);
    } else if (in.kind == DN_BEGIN) {
#pragma unroll
      for (int l = 0; l < NLV; ++l)
        if (l == in.level) {
          for (int i = 0; i < Q; ++i) acc[l][i] = T(0);
          if (l > 0 && in.op >= 0) apply(acc[l], acc[l > 0 ? l - 1 : 0], in.op);
        }
    } else {
      gbl<T>* Y = as_global(data) + (int64_t(in.box) + store_shift) * box_stride;
#pragma unroll
      for (int l = 0; l < NLV; ++l)
        if (l == in.level && ok)
          for (int i = 0; i < Q; ++i) store_stream(Y + int64_t(i) * ncol + col, acc[l][i]);
    }
  }
}

// --------------------------------------------------------------------------
// The whole tree of a column group in LDS (M2M, M2L and L2L, Eqs. 11-13 and
// 17a-c) on chains: trees split along x only whose every level is one
// unbroken row of boxes, and whose every interaction list is the in-range
// part of one displacement stencil per level and x parity.
// Displacements on the x axis keep the four reflection classes of the real
// components apart, so each class is a problem of its own.  One block per
// (group of C carried columns, class CLS) reads the leaf multipoles of its
// columns once, runs the upward levels and then the downward levels in LDS,
// and writes the leaf local expansions once: per j batch HBM sees one read
// and one write of the leaf rows, where the walks and level passes write and
// read back every box of the tree.
//
// LDS holds the class's NK components of every box slot and column at
// lds[(slot * NK + k) * C + c].  At each level the threads take the level's
// (box, column) items, two at a time; on the downward levels one half of the
// threads takes the boxes of even x and the other half those of odd x, so
// that the operators of a wave are uniform and come from scalar loads.  A
// downward level's local expansions replace its multipoles once all are
// formed (held in registers across a barrier).  Each box takes its terms in the order of
// the level-by-level passes (parent first, then the stencil in increasing
// displacement; out-of-range stencil entries are skipped) with FP64
// operators and accumulators.
// --------------------------------------------------------------------------
constexpr int kChainStencil = 8;   // stencil entries per parity
struct ChainLevel {
  int32_t n, slot0, x0, pad0;     // boxes of the level, first box slot, x index of the first box
  int32_t up_op[2];               // M2M operators of the even-x and odd-x child (levels above the leaves)
  int32_t dn_op[2];               // L2L operators of even-x and odd-x boxes (levels below the first)
  int32_t ne[2];                  // stencil entries of even-x and odd-x boxes
  int32_t d[2][kChainStencil];    // source minus target, increasing
  int32_t op[2][kChainStencil];   // M2L operator of each entry
  int32_t pad[6];
};
constexpr int kTreeThreads = 512;
constexpr int kTreeMaxBoxes = 512;  // box slots in LDS
constexpr int kTreeRounds = 4;      // (box, column) items per thread on a downward level above the leaves (even)

__host__ __device__ constexpr int class_size(int Q, int sym, int cls) {
  int n = 0;
  for (int q = 0; q < Q; ++q) n += real_class(q, sym) == cls ? 1 : 0;
  return n;
}
// the class's components in ascending q, 4 bits each
__host__ __device__ constexpr uint64_t class_pack(int Q, int sym, int cls) {
  uint64_t p = 0;
  int k = 0;
  for (int q = 0; q < Q; ++q)
    if (real_class(q, sym) == cls) p |= uint64_t(q) << (4 * k++);
  return p;
}
// columns per block: 64 bytes per component row of a box slot
__host__ __device__ constexpr int tree_cols(int tbytes) { return 64 / tbytes; }

template <class T, int CLS>
__global__ __launch_bounds__(kTreeThreads) void tree_chain_kernel(
    T* __restrict__ data, int64_t box_stride, ColMap cm, const ChainLevel* __restrict__ lv, int nlev,
    const double* __restrict__ opc, int32_t leaf0, int32_t nleaf, int32_t nbox, int64_t load_shift,
    int64_t store_shift, int64_t ngroups) {
  constexpr int Q = 9, SYM = 1;
  constexpr int NK = class_size(Q, SYM, CLS);
  constexpr uint64_t QP = class_pack(Q, SYM, CLS);
  constexpr int C = tree_cols(int(sizeof(T)));
  constexpr int NT = kTreeThreads;
  static_assert(NK > 0 && NT % C == 0, "class layout");
  __shared__ T lds[kTreeMaxBoxes * NK * C];
  const int64_t per = (int64_t(gridDim.x) + 7) / 8;
  const int64_t grp = int64_t(blockIdx.x % 8) * per + blockIdx.x / 8;
  if (grp >= ngroups) return;
  const int tid = threadIdx.x;
  const int c = tid % C;
  const int64_t v = grp * C + c;
  const bool ok = v < cm.nvalid;
  const int64_t col = ok ? carried_col(cm, v) : 0;   // invalid columns read column 0, store nothing
  const int64_t ncol = cm.ncol;
  auto comp = [](int k) { return int((QP >> (4 * k)) & 15); };
  // leaf multipoles of the class into LDS, rows r = (leaf, k), U loads in flight per thread
  {
    const gbl<const T>* base = as_global(static_cast<const T*>(data)) + col;
    constexpr int RPP = NT / C;   // rows per pass
    constexpr int U = 16;
    const int nrow = nleaf * NK;
    for (int r0 = tid / C; r0 < nrow; r0 += U * RPP) {
      T x[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int r = r0 + u * RPP;
        if (r < nrow) {
          const int b = r / NK, k = r - b * NK;
          x[u] = base[(int64_t(leaf0 + b) + load_shift) * box_stride + int64_t(comp(k)) * ncol];
        }
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int r = r0 + u * RPP;
        if (r < nrow) lds[(int(leaf0) * NK + r) * C + c] = x[u];
      }
    }
  }
  __syncthreads();
  const cst<double>* A0 = as_const(opc);
  const cst<ChainLevel>* LV = as_const(lv);   // uniform fields, read where used (scalar loads)
  // Two items (box, column) per thread go through the terms together: one
  // operator read serves both, and their LDS reads and FMA chains overlap.
  // acc_r += T_op x(slot_r) over the class (T[i][k] at A[i * NK + k]); an
  // item that does not take the term reads slot `alt` and adds exact zeros.
  auto term2 = [&](double (&a0)[NK], double (&a1)[NK], int op, int sl0, bool t0, int sl1, bool t1, int alt) {
    const cst<double>* A = A0 + op * (NK * NK);
    const int u0 = t0 ? sl0 : alt, u1 = t1 ? sl1 : alt;
    double x0[NK], x1[NK];
#pragma unroll
    for (int k = 0; k < NK; ++k) {
      x0[k] = t0 ? double(lds[(u0 * NK + k) * C + c]) : 0.0;
      x1[k] = t1 ? double(lds[(u1 * NK + k) * C + c]) : 0.0;
    }
#pragma unroll
    for (int i = 0; i < NK; ++i)
#pragma unroll
      for (int k = 0; k < NK; ++k) {
        const double a = A[i * NK + k];
        a0[i] = fma(a, x0[k], a0[i]);
        a1[i] = fma(a, x1[k], a1[i]);
      }
  };
  // upward levels: Omega(p) = sum over the children present (x = 2 x_p, 2 x_p + 1) of T Omega(child)
  for (int li = nlev - 2; li >= 0; --li) {
    const cst<ChainLevel>& L = LV[li];
    const cst<ChainLevel>& Lc = LV[li + 1];
    const int n = L.n, s0 = L.slot0, x0 = L.x0, cn = Lc.n, cs0 = Lc.slot0, cx0 = Lc.x0;
    for (int it = tid; it < n * C; it += 2 * NT) {
      const bool v1 = it + NT < n * C;
      const int p0 = it / C, p1 = v1 ? (it + NT) / C : p0;
      const int c0 = 2 * (x0 + p0) - cx0, c1 = 2 * (x0 + p1) - cx0;   // indices of the even-x children
      double a0[NK], a1[NK];
#pragma unroll
      for (int k = 0; k < NK; ++k) a0[k] = a1[k] = 0.0;
      term2(a0, a1, L.up_op[0], cs0 + c0, c0 >= 0 && c0 < cn, cs0 + c1, c1 >= 0 && c1 < cn, cs0);
      term2(a0, a1, L.up_op[1], cs0 + c0 + 1, c0 + 1 >= 0 && c0 + 1 < cn, cs0 + c1 + 1, c1 + 1 >= 0 && c1 + 1 < cn,
            cs0);
#pragma unroll
      for (int k = 0; k < NK; ++k) {
        lds[((s0 + p0) * NK + k) * C + c] = T(a0[k]);
        if (v1) lds[((s0 + p1) * NK + k) * C + c] = T(a1[k]);
      }
    }
    __syncthreads();
  }
  // downward levels: Mloc(b) = T_dn Mloc(parent) + sum over the stencil of T Omega(b + d);
  // out-of-range stencil entries add exact zeros (the order of the real terms is kept).
  // The first half of the threads takes the boxes of even x, the second half
  // those of odd x (each wave one parity: uniform operators).
  constexpr int NH = NT / 2;
  const int par = __builtin_amdgcn_readfirstlane(tid / NH), ht = tid % NH;
  for (int li = 0; li < nlev; ++li) {
    const cst<ChainLevel>& L = LV[li];
    const int n = L.n, s0 = L.slot0, x0 = L.x0;
    const int ps0 = li > 0 ? int(LV[li - 1].slot0) : 0, px0 = li > 0 ? int(LV[li - 1].x0) : 0;
    const int b0 = (par - x0) & 1, cnt = (n - b0 + 1) / 2, nit = cnt * C;
    const int ne = L.ne[par], dop = L.dn_op[par];
    // the items it and it + NH of this parity; v1: the second one exists
    auto items = [&](int it, bool v1, int& b0_, int& b1_, double (&a0)[NK], double (&a1)[NK]) {
      b0_ = b0 + 2 * (it / C);
      b1_ = v1 ? b0 + 2 * ((it + NH) / C) : b0_;
#pragma unroll
      for (int k = 0; k < NK; ++k) a0[k] = a1[k] = 0.0;
      if (li > 0)
        term2(a0, a1, dop, ps0 + ((x0 + b0_) >> 1) - px0, true, ps0 + ((x0 + b1_) >> 1) - px0, true, 0);
#pragma unroll 1
      for (int e = 0; e < ne; ++e) {
        const int d = L.d[par][e], op = L.op[par][e];
        const int q0 = b0_ + d, q1 = b1_ + d;
        term2(a0, a1, op, s0 + q0, q0 >= 0 && q0 < n, s0 + q1, q1 >= 0 && q1 < n, s0);
      }
    };
    if (li == nlev - 1) {   // leaves: the local expansions to HBM
      for (int it = ht; it < nit; it += 2 * NH) {
        const bool v1 = it + NH < nit;
        int bb0, bb1;
        double a0[NK], a1[NK];
        items(it, v1, bb0, bb1, a0, a1);
        if (ok) {
          gbl<T>* Y0 = as_global(data) + (int64_t(nbox) + s0 + bb0 + store_shift) * box_stride + col;
          gbl<T>* Y1 = as_global(data) + (int64_t(nbox) + s0 + bb1 + store_shift) * box_stride + col;
#pragma unroll
          for (int k = 0; k < NK; ++k) {
            store_stream(Y0 + int64_t(comp(k)) * ncol, T(a0[k]));
            if (v1) store_stream(Y1 + int64_t(comp(k)) * ncol, T(a1[k]));
          }
        }
      }
    } else {   // at most kTreeRounds items per thread (checked on the host), two at a time
      T hold[kTreeRounds][NK];
      int hs[kTreeRounds];
#pragma unroll
      for (int q = 0; q < kTreeRounds; q += 2) {
        const int it = ht + q * NH;
        hs[q] = hs[q + 1] = -1;
        if (it < nit) {
          const bool v1 = it + NH < nit;
          int bb0, bb1;
          double a0[NK], a1[NK];
          items(it, v1, bb0, bb1, a0, a1);
          hs[q] = s0 + bb0;
          if (v1) hs[q + 1] = s0 + bb1;
#pragma unroll
          for (int k = 0; k < NK; ++k) {
            hold[q][k] = T(a0[k]);
            hold[q + 1][k] = T(a1[k]);
          }
        }
      }
      __syncthreads();   // the level's multipoles are read no more
#pragma unroll
      for (int q = 0; q < kTreeRounds; ++q)
        if (hs[q] >= 0)
#pragma unroll
          for (int k = 0; k < NK; ++k) lds[(hs[q] * NK + k) * C + c] = hold[q][k];
    }
    __syncthreads();
  }
}

// Operators of every reflection class in compact form for tree_chain_kernel:
// class c of op o at out[off_c + (o * n_c + i) * n_c + k] = T[q_i][q_k]
// (q_i the class's components in ascending order, off_c the sum of
// nops * n_c'^2 over the classes before c).  One thread per element; Q <= 16
// (one row tile of the fragment-ordered operator).
static __global__ void opclass_kernel(const double* __restrict__ ops, int nops, int Q, int sym, double* __restrict__ out) {
  const int KS = ksteps_of(Q);
  const int ncls = sym == 1 ? 4 : sym == 2 ? 2 : 1;
  int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  for (int cl = 0; cl < ncls; ++cl) {
    const int n = class_size(Q, sym, cl);
    const int64_t sz = int64_t(nops) * n * n;
    if (e < sz) {
      const int o = int(e / (n * n)), r = int(e % (n * n));
      const int i = r / n, k = r % n;
      int qi = -1, qk = -1;
      for (int q = 0, m = 0; q < Q; ++q)
        if (real_class(q, sym) == cl) {
          if (m == i) qi = q;
          if (m == k) qk = q;
          ++m;
        }
      out[e] = ops[int64_t(o) * KS * 64 + (qk >> 2) * 64 + qi + 16 * (qk & 3)];
      return;
    }
    e -= sz;
    out += sz;
  }
}

// out[r*ldo + c] = float(in[r*ldi + c]) for r < rows, c < cols
static __global__ void to_float_kernel(const double* __restrict__ in, int64_t ldi, float* __restrict__ out, int64_t ldo,
                                int64_t rows, int64_t cols) {
  const int64_t n = rows * cols;
  for (int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; e < n; e += int64_t(gridDim.x) * blockDim.x) {
    const int64_t r = e / cols, c = e % cols;
    out[r * ldo + c] = float(in[r * ldi + c]);
  }
}

// K[r, i0 + i] = (acc ? K : 0) + sum_{e in occ(r)} KB[row_e, i]   (fixed order)
__device__ inline void reduce_elem(const double* __restrict__ KB, int64_t ni, const int32_t* __restrict__ occ_ptr,
                                   const int32_t* __restrict__ occ_row, double* __restrict__ K, int64_t ldk, int i0,
                                   int accumulate, int r, int64_t i) {
  double s = 0.0;
  const gbl<const int32_t>* op = as_global(occ_ptr);
  const gbl<const int32_t>* orow = as_global(occ_row);
  const gbl<const double>* kb = as_global(KB);
  for (int e = op[r]; e < op[r + 1]; ++e) s += kb[int64_t(orow[e]) * ni + i];
  gbl<double>* k = as_global(K) + int64_t(r) * ldk + i0 + i;
  *k = accumulate ? *k + s : s;
}

static __global__ __launch_bounds__(256) void reduce_kernel(const double* __restrict__ KB, int64_t ni,
                                                     const int32_t* __restrict__ occ_ptr,
                                                     const int32_t* __restrict__ occ_row, double* __restrict__ K,
                                                     int64_t ldk, int i0, int accumulate) {
  const int r = blockIdx.y;
  const int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (i >= ni) return;
  reduce_elem(KB, ni, occ_ptr, occ_row, K, ldk, i0, accumulate, r, i);
}

static __global__ void zero_cols_kernel(double* __restrict__ K, int64_t ldk, int i0, int64_t ni) {
  const int r = blockIdx.y;
  const int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (i < ni) K[int64_t(r) * ldk + i0 + i] = 0.0;
}

}  // namespace occk
