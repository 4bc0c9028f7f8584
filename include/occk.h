/*
 * occk — far-field occupied exchange K^ff_ri of occ-FMM-K on AMD MI355X (gfx950).
 *
 * Method: Le & Shiozaki, "Occupied-orbital fast multipole method for efficient
 * exact exchange evaluation" (arXiv:1708.05353), Theory section:
 *   K_ri = 2 sum_j (rj|ji)                                   Eq. (5)
 *   O^{rj,X} = sum_s O^{rs,X} C_sj,  O^{ij,X} = sum_r O^{rj,X} C_ri   Eq. (15a,b)
 *   upward / interaction-list / downward translations per (i,j)    Eq. (17a-c)
 *   K^ff_ri = 2 sum_X sum_j sum_lm O^{rj,X}_lm Mloc^{ij}_lm(X)      Eq. (18)
 * with the scaled solid harmonics of Eq. (4a,b), AO multipoles of Eq. (8)
 * about the centre of the leaf box that holds each AO pair, and square
 * truncation l, l' <= L.
 *
 * Conventions for every entry point
 *   - Return value: OCCK_OK (0) or a negative OCCK_E* code; occk_last_error()
 *     then returns a thread-local message.  No C++ exception crosses the ABI.
 *   - All argument validation happens on the host before any HIP call.
 *   - Pointers documented as "device" must be HIP device allocations on the
 *     current device; "host" pointers are ordinary host memory.
 *   - A tree handle is used from one host thread / one stream at a time.
 */
#ifndef OCCK_H
#define OCCK_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define OCCK_ABI_VERSION 1

enum {
  OCCK_OK = 0,
  OCCK_EINVAL = -1,      /* bad argument (null, out of range, inconsistent)   */
  OCCK_ENOMEM = -2,      /* host or device allocation failed / over the cap   */
  OCCK_EHIP = -3,        /* a HIP runtime call failed                          */
  OCCK_EHANDLE = -4,     /* freed, forged or foreign handle                    */
  OCCK_ENONFINITE = -5,  /* non-finite input where finite values are required  */
  OCCK_ESTATE = -6       /* operation not valid in the handle's current state  */
};

/* Arithmetic of the contractions.  Translation operators are always generated
 * in FP64 (then rounded for the mixed modes) and the per-leaf K partials and K
 * are always accumulated in FP64.
 *   FP64    every contraction on FP64 MFMA
 *   FP32    FP32 operands, FP32 MFMA, FP32 accumulation
 *   BF16X3  half/Omega/L2P as split-BF16 products hi*hi + hi*lo + lo*hi with
 *           FP32 accumulation (~2^-16 per product); translations on FP32 MFMA.
 *           Outside the 1e-6 target of the mixed path: its bound is 5e-5
 *           (normwise errors of 4e-6 to 9e-6 on the test systems)
 *   BF16X6  three-way split, six products (~2^-24 per product); translations
 *           on FP32 MFMA
 * The FP32 translations at L >= 3 accumulate a box's interaction list in FP32:
 * on large 3-D trees at high rank (a 6187-function globule at L = 8) FP32 and
 * BF16X6 reach ~5e-6 against FP64 instead of 1e-6. */
enum { OCCK_PREC_FP64 = 0, OCCK_PREC_FP32 = 1, OCCK_PREC_BF16X3 = 2, OCCK_PREC_BF16X6 = 3 };
enum { OCCK_RANK_FIXED = 0, OCCK_RANK_LEARNED = 1 };

/* Molecular system: atoms and uncontracted normalised Cartesian Gaussian
 * primitive shells (l = 0 or 1).  Functions are numbered shell by shell; a p
 * shell contributes x, y, z in that order.  Coordinates in bohr.  All arrays
 * are host memory owned by the caller and only read during occk_build_tree. */
typedef struct occk_system {
  int32_t natoms;
  const double* xyz;          /* [natoms*3] */
  int32_t nshell;
  const int32_t* shell_atom;  /* [nshell], 0 <= atom < natoms */
  const int32_t* shell_l;     /* [nshell], 0 or 1 */
  const double* shell_exp;    /* [nshell], > 0 */
} occk_system;

/* Box-tree parameters (Theory section: hierarchy, near/far split).
 *   split_mask  bit0 x, bit1 y, bit2 z: dimensions that are subdivided
 *   depth       number of subdivisions (2^depth boxes per split dimension), 1..12
 *   ws          two boxes of one level are near iff the Chebyshev distance of
 *               their integer indices is <= ws (0..4)
 *   lmax        multipole rank L (0..15); l <= L and l' <= L.  The exchange
 *               entry points take L <= 8; occk_far_J takes any rank
 *   pair_log_thresh  keep an ordered shell pair iff (ab/(a+b))|A-B|^2 <= thresh
 *               (+inf keeps every pair)
 * Root box: over the split dimensions E = largest extent of the pair centres,
 * delta = 0.05 E + 1, lo = min - 0.35 delta, width W = E + delta; a dimension
 * that is not split is one layer centred on the midpoint of the pair centres.
 * The interaction list of a box holds the non-near boxes of its level whose
 * parents are near its parent; empty boxes are pruned.
 *   near_rule   OCCK_NEAR_BOXES: near iff the box-index distance is <= ws (above);
 *               OCCK_NEAR_EXTENT: the paper's criterion by extents (Theory
 *               section, the near/far paragraph): a pair distribution of
 *               exponent p = a + b has extent erfc^-1(ext_tau)/sqrt(p); a box's
 *               extent is the largest |P - X_box| + extent over the
 *               distributions it holds; two boxes of one level are far iff
 *               |X_a - X_b| > (1 + ext_ws)(ext_a + ext_b); near lists are
 *               formed top down (ws is then unused)
 *   ext_ws      slack of the extent rule (the paper's ws; 0 typical), -1 < ext_ws <= 10
 *   ext_tau     extent threshold, 0 < ext_tau < 0.5 (1e-8: the s-type
 *               penetration erfc of two separated distributions stays below it) */
enum { OCCK_NEAR_BOXES = 0, OCCK_NEAR_EXTENT = 1 };
typedef struct occk_tree_params {
  int32_t split_mask;
  int32_t depth;
  int32_t ws;
  int32_t lmax;
  double pair_log_thresh;
  int32_t near_rule;
  double ext_ws;
  double ext_tau;
} occk_tree_params;

typedef struct occk_tree occk_tree;
typedef struct occk_selector occk_selector;
typedef struct occk_batch occk_batch;

#define OCCK_MAX_LEVELS 13

typedef struct occk_tree_info_t {
  int32_t nbasis;
  int32_t lmax;
  int32_t ncomp;               /* (L+1)^2 real components per box            */
  int32_t depth;
  int32_t lmin;                /* coarsest level with a non-empty interaction
                                  list, -1 when there is no far field        */
  int32_t nleaf;
  int32_t nbox;                /* boxes on levels lmin..depth                */
  int32_t boxes_per_level[OCCK_MAX_LEVELS];
  int32_t il_per_level[OCCK_MAX_LEVELS];
  int64_t n_il;                /* ordered interaction-list pairs, all levels */
  int64_t n_edges;             /* parent-child edges between lmin and depth  */
  int64_t npairs;              /* screened ordered AO function pairs         */
  int64_t sum_nb;              /* sum over leaves of functions in the leaf   */
  int64_t sum_nb2;             /* sum over leaves of nB^2                    */
  int32_t max_nb;
  int32_t n_ops;               /* translation operators generated per call   */
  int64_t m2m_nnz;             /* structural nonzeros of one real-form M2M
                                  (= L2L) operator                           */
  double lo[3], width, mid[3];
  int64_t n_near;              /* ordered near leaf pairs (the near field), self pairs included */
} occk_tree_info_t;

typedef struct occk_far_opts {
  int32_t precision;           /* OCCK_PREC_*                                  */
  int32_t rank_mode;           /* OCCK_RANK_*; LEARNED needs a live selector  */
  const occk_selector* selector;
  int32_t jblock;              /* occupied j columns per batch, 0 = automatic:
                                  the widest batch (<= 256; <= 128 where an FP64
                                  call runs the two-stream schedule) whose
                                  workspace fits the device-byte cap          */
  int32_t accumulate;          /* 0: K[:, i0:i1] = K^ff, 1: K[:, i0:i1] += K^ff */
  double pair_thresh;          /* occupied-pair screening for localised orbitals
                                  (Conclusion: localised orbitals and screening of
                                  occupied pairs), 0 = off.  With n_Ai the sum of
                                  |C_ti| over the functions t centred in leaf A
                                  and W_AA' the largest Gaussian product factor
                                  exp(-ab/(a+b)|A-B|^2) of a screened function
                                  pair with one function centred in A and the
                                  other in A', the pair (i, j) is kept when
                                  b_ij = sum_(A,A') n_Aj W_AA' n_A'i >= pair_thresh
                                  (b_ij bounds sum over screened pairs (t, u) of
                                  their factor times |C_tj| |C_ui|).  A j batch
                                  then carries i only up to the last kept i of
                                  its j (orbitals ordered along the system make
                                  this a band), so every pair inside the band is
                                  evaluated, kept or not.  Needs i0 == j0 and
                                  i1 == j1; synchronises the stream once per call */
  int32_t one_stream;          /* 0: when the i and j ranges coincide and the tree
                                  runs its downward translations as walks, the
                                  L2P of each j batch runs on a second stream of
                                  the library, overlapping the next batch's Omega
                                  and translations (the call still completes in
                                  order on hip_stream); 1: everything on
                                  hip_stream, one kernel at a time (kernel
                                  timings, profiles) */
  int32_t lds_tree;            /* 1: on chains (trees split along x whose levels are
                                  unbroken rows of boxes, Q = 9) run the
                                  translations of a j batch (Eqs. 17a-c) as one
                                  kernel per reflection class that holds the
                                  whole tree of a group of columns in LDS and
                                  moves only leaf rows through HBM; other trees
                                  keep the walks and level passes.  0 (default):
                                  subtree walks and level-by-level passes, which
                                  are faster on the chains measured */
} occk_far_opts;

/* Returns OCCK_ABI_VERSION. */
int32_t occk_abi_version(void);

/* Thread-local message describing the last non-zero status; never NULL. */
const char* occk_last_error(void);

/* Step 1 of the method (per geometry, host only, no HIP call): screened AO
 * pairs and their Gaussian-product centres, pair -> leaf assignment, the box
 * levels, neighbour and interaction lists (Theory section), and the leaf AO
 * multipole integrals of Eq. (8) in FP64 about each leaf centre.  Everything
 * needed is copied; *out owns it.  Device memory is allocated lazily by the
 * first occk_far_K.  Errors: EINVAL (bad system/params, a pair centre within
 * 1e-8 h of a leaf boundary, a screening value within 1e-9 of the threshold),
 * ENOMEM. */
int32_t occk_build_tree(const occk_system* sys, const occk_tree_params* params, occk_tree** out);

/* Frees host and device memory of the handle; NULL is accepted.  EHANDLE for
 * a handle that is not live. */
int32_t occk_free_tree(occk_tree* tree);

/* Counts of the built tree (host only). */
int32_t occk_tree_info(const occk_tree* tree, occk_tree_info_t* info);

/* Algorithmic flop model of one occk_far_K call over ni output columns i and
 * nj summed columns j (host only).  The terms are the method's own work on the
 * built tree, Q = (L+1)^2:
 *   half   Eq. (15a)  2 Q nj npairs
 *   omega  Eq. (15b)  2 Q ni nj sum_B nB, or Q n (n+1) sum_B nB when symmetric
 *   m2m    Eq. (17a)  2 z nc E   (z = m2m_nnz, E = n_edges)
 *   m2l    Eq. (17b)  2 Q^2 nc n_il
 *   l2l    Eq. (17c)  2 z nc E
 *   l2p    Eq. (18)   2 Q ni nj sum_B nB
 * with nc = ni nj translated (j, i) columns, or nc = n (n+1)/2 when symmetric
 * != 0: the occupied-pair multipoles and every translated expansion are
 * symmetric in (i, j), so that many columns are all the method must carry
 * (symmetric needs ni == nj = n; EINVAL otherwise).  A tree with no far field
 * gives zeros.  out->total is the sum of the six terms. */
typedef struct occk_flops_t {
  int64_t half, omega, m2m, m2l, l2l, l2p, total;
} occk_flops_t;
int32_t occk_tree_flops(const occk_tree* tree, int32_t ni, int32_t nj, int32_t symmetric, occk_flops_t* out);

/* Host-side export for checking the tree against an independent one.
 *   leaf_coords  [nleaf*3] int32 integer box indices of the leaves (level depth),
 *                in the library's leaf order; may be NULL
 *   il_level, il_target, il_source  [n_il] int32: level and the integer
 *                box-index triples are not exported; instead target and source
 *                are leaf-order-independent linear keys x + 4096 (y + 4096 z)
 *                of the boxes at that level; may be NULL
 *   pair_leaf    [npairs] int32 leaf index of each screened pair in the order
 *                (shell a, shell b, function of a, function of b) with a, b
 *                ascending; may be NULL */
int32_t occk_tree_export(const occk_tree* tree, int32_t* leaf_coords, int32_t* il_level,
                         int32_t* il_target, int32_t* il_source, int32_t* pair_leaf);

/* Host export of the near field: for every leaf (library order), the sorted
 * leaves near it, itself included, as CSR: ptr [nleaf+1], idx [n_near]
 * (tree_info).  Either may be NULL. */
int32_t occk_tree_near(const occk_tree* tree, int32_t* ptr, int32_t* idx);

/* Host copy of one leaf's data: its sorted function list (nb entries) and the
 * dense real-form AO multipole block O[q][a][b] (q over (L+1)^2 real
 * components: (l,0), then Re and Im of (l,m) for m = 1..l; a, b local
 * function indices) about the leaf centre, Eq. (8).  Either output may be NULL.
 * *nb receives the function count.  Host only. */
int32_t occk_tree_leaf(const occk_tree* tree, int32_t leaf, int32_t* nb, int32_t* funcs, double* O);

/* Far-field occupied exchange, Eqs. (15)-(18), on the GPU:
 *   K[r, i] = 2 sum_{j in [j0,j1)} (rj|ji)_ff   for i in [i0, i1), all r
 * C: device, row-major nbasis x ldc FP64, columns 0..nocc-1 are the occupied
 *    orbitals (ldc >= nocc).  Only columns in [i0,i1) and [j0,j1) are read.
 * K: device, row-major nbasis x ldk FP64 (ldk >= i1); columns outside
 *    [i0,i1) are not touched.  K must not overlap C.
 * opts: NULL means FP64, fixed rank, automatic j batching, overwrite.
 * hip_stream: hipStream_t (NULL = default stream).  All work is enqueued
 *    asynchronously on it; the caller synchronises.  The first call on a
 *    handle uploads the tree and allocates the workspace (synchronous).
 * Errors (before any device work): EINVAL for null/ill-formed arguments or
 *    ranges (0 <= i0 <= i1 <= nocc, 0 <= j0 <= j1 <= nocc), EHANDLE, ESTATE
 *    (LEARNED without a trained selector), ENOMEM (workspace beyond
 *    OCCK_MAX_DEVICE_BYTES or hipMalloc failure), EHIP. */
int32_t occk_far_K(occk_tree* tree, const double* C, int64_t ldc, int32_t nocc,
                   int32_t i0, int32_t i1, int32_t j0, int32_t j1,
                   const occk_far_opts* opts, double* K, int64_t ldk, void* hip_stream);

/* Allocation-free variant of occk_far_K, for callers that cannot allocate
 * device memory: code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc.  Same arguments, result and errors as
 * occk_far_K, within these limits:
 *   - FP64 and fixed rank only (EINVAL otherwise);
 *   - the tree's device copy must exist: the handle's first occk_far_K makes
 *     it (ESTATE before that; EINVAL when it is on another device);
 *   - the workspace (box expansions, half-transformed multipoles, per-leaf K
 *     partials, GEMM tile tables) is placed in one fixed device region of
 *     OCCK_NOALLOC_SCRATCH_BYTES per GPU, a static device array held from
 *     the library's loading until the process ends; jblock = 0 takes the
 *     widest j batch (<= 256) whose workspace fits; ENOMEM, with the sizes in
 *     the message, when an explicit jblock does not fit or the workspace of a
 *     one-column batch does not;
 *   - it synchronises hip_stream on entry, copies the tile tables into the
 *     region with hipMemcpy, and calls neither hipMalloc nor hipFree;
 *   - every call on one GPU uses the same region, which keeps the last
 *     call's contents (nothing in it has to start at zero): calls that
 *     overlap in time on one GPU (other streams or threads) race, and the
 *     caller must serialise them.
 * The handle's own workspace (that of occk_far_K) is left as it was. */
#define OCCK_NOALLOC_SCRATCH_BYTES (128ll << 20)
int32_t occk_far_K_noalloc(occk_tree* tree, const double* C, int64_t ldc, int32_t nocc,
                           int32_t i0, int32_t i1, int32_t j0, int32_t j1,
                           const occk_far_opts* opts, double* K, int64_t ldk, void* hip_stream);

/* Far-field Coulomb matrix on the GPU, through the same tree (Theory section:
 * the Coulomb passage with Eq. 10 and the J^ff formula after it):
 *   O^B_lm    = sum over the pairs (t,u) of leaf B of D_tu O^{tu,B}_lm
 *   Mloc_lm(X) = (-1)^l sum_far sum M_{l+l',m+m'}(X - X') O^{X'}_{l'm'}, by
 *               upward (Eq. 11), interaction-list (Eq. 12) and downward
 *               (Eq. 13) translations of that single column
 *   J[r, s]   = sum_lm O^{rs,X}_lm Mloc_lm(X) for every screened pair (r,s)
 *               of every leaf X (the pair's own leaf)
 * at the tree's rank L (the paper's L^J = 10 for Coulomb; trees of any rank
 * up to 15).  FP64 throughout.
 * D: device, row-major nbasis x ldd FP64, the density matrix (only the
 *    entries D[t, u] of screened pairs are read); ldd >= nbasis.
 * J: device, row-major nbasis x ldj FP64; accumulate = 0: J = J^ff with zeros
 *    outside the screened pairs; accumulate = 1: J[r, s] += J^ff_rs at the
 *    screened pairs only.  J must not overlap D.
 * Asynchronous on hip_stream; the first call on a handle uploads the pair
 * multipoles and the tables (synchronous).  Errors: EINVAL, EHANDLE, ENOMEM
 * (beyond OCCK_MAX_DEVICE_BYTES, checked before any HIP call), EHIP. */
int32_t occk_far_J(occk_tree* tree, const double* D, int64_t ldd, double* J, int64_t ldj,
                   int32_t accumulate, void* hip_stream);

/* Near-field occupied exchange with exact integrals over the s/p primitives
 * (Theory section: the distributions whose leaf boxes are near are not
 * expanded; with the exchange definition of the Introduction):
 *   K[r, i] (+)= 2 sum_j sum_{(r,s) in B, (t,u) in B'} (rs|tu) C_sj C_tj C_ui
 * over the ordered pairs of leaves B, B' that are near (B = B' included;
 * the leaf-level near relation of the tree's near_rule), i.e.
 * K = X C with X_ru = sum_{s,t} (rs|tu) D_st, D = 2 C C^T.  Together with
 * occk_far_K it gives the whole exchange.  Integrals: McMurchie-Davidson
 * over the screened shell pairs, FP64; X is accumulated with atomic adds, so
 * the last bits may differ between runs.
 * C: device, row-major nbasis x ldc FP64 (ldc >= nocc; all nocc columns are
 *    the occupied orbitals).  K: device, row-major nbasis x ldk FP64 (ldk >=
 *    nocc); accumulate = 0: K[:, :nocc] = K^nf, 1: K[:, :nocc] += K^nf.  K must
 *    not overlap C.
 * The first call on a handle (or with another nocc) builds the shell-pair
 * tables and allocates D, X and C^T on the device (3 nbasis^2-sized FP64
 * buffers at most; checked against OCCK_MAX_DEVICE_BYTES before any HIP
 * call).  Asynchronous on hip_stream.  Errors: EINVAL, EHANDLE, ENOMEM, EHIP. */
int32_t occk_near_K(occk_tree* tree, const double* C, int64_t ldc, int32_t nocc, double* K, int64_t ldk,
                    int32_t accumulate, void* hip_stream);

/* Work of the handle's near-field tables: wave tasks and shell quartets per
 * occk_near_K call (either pointer may be NULL).  ESTATE before the first call. */
int32_t occk_near_info(occk_tree* tree, int64_t* tasks, int64_t* quartets);

/* Algorithmic flop model of one occk_far_J call (host only), Q = (L+1)^2:
 *   dens  2 Q npairs     density-contracted leaf multipoles
 *   m2m   2 z E          upward (z = m2m_nnz, E = n_edges)
 *   m2l   2 Q^2 n_il     interaction lists
 *   l2l   2 z E          downward
 *   pair  2 Q npairs     J_rs from the leaf's local expansion
 * A tree with no far field gives zeros. */
typedef struct occk_jflops_t {
  int64_t dens, m2m, m2l, l2l, pair, total;
} occk_jflops_t;
int32_t occk_tree_flops_J(const occk_tree* tree, occk_jflops_t* out);

/* The band of the handle's last occk_far_K with pair_thresh > 0 (host only):
 * *carried = the (j, i) columns it carried through the translations,
 * *jblock = its j batch width, *nband = its number of j batches, and
 * band_end[k] (k < min(cap, *nband)) = the end (exclusive, relative to i0)
 * of the i range carried by batch k, whose j are [k jblock, (k+1) jblock)
 * relative to j0.  Zeros before such a call.  band_end may be NULL when
 * cap is 0; the other pointers must be valid.  OCCK_EINVAL for a NULL
 * pointer or negative cap. */
int32_t occk_pair_screen_info(occk_tree* tree, int64_t* carried, int32_t* jblock, int32_t* band_end, int32_t cap,
                              int32_t* nband);

/* Workspace of the handle's last occk_far_K: the j batch width used (-1
 * before the first call) and the device bytes held by the handle.  Either
 * pointer may be NULL. */
int32_t occk_workspace_info(occk_tree* tree, int32_t* jblock, int64_t* bytes);

/* ---- many systems in one persistent launch ---- */

/* Plan for evaluating K^ff of nsys independent systems (all i, all j of
 * each) in one persistent (cooperative) kernel launch: the same steps as
 * occk_far_K (Eqs. 15-18, operator generation and operand conversion
 * included, the symmetric schedule over j batches) become tasks grouped by
 * stage; the blocks share the tasks of a stage and meet at a grid barrier
 * between stages.  trees: live handles with a far field and a common lmax;
 * the plan keeps pointers to them (free the plan first); lmax up to 8, as for
 * occk_far_K.  nocc[k]: occupied
 * count of system k.  opts: precision (any OCCK_PREC_*); rank_mode must be
 * FIXED; jblock: j batch width of every system (0: chosen per system as in
 * occk_far_K; capped at nocc); accumulate is ignored (K is overwritten).
 * Uploads the trees and allocates every workspace (synchronous).  Errors:
 * EINVAL, EHANDLE, ENOMEM, EHIP. */
int32_t occk_batch_create(int32_t nsys, occk_tree* const* trees, const int32_t* nocc, const occk_far_opts* opts,
                          occk_batch** out);

/* One persistent cooperative launch on hip_stream.
 * C[k]: device, row-major nbasis_k x ldc[k] FP64 (ldc[k] >= nocc[k]);
 * K[k]: device, row-major nbasis_k x ldk[k] FP64, columns 0..nocc[k]-1 are
 * overwritten with K^ff.  Asynchronous.  Calls on one plan must not overlap
 * (they share the workspaces).  A standalone occk_far_K on one of the trees
 * replaces its workspace; the next run rebuilds the plan's tables
 * (synchronously). */
int32_t occk_batch_run(occk_batch* plan, const double* const* C, const int64_t* ldc, double* const* K,
                       const int64_t* ldk, void* hip_stream);

/* Autotuner: runs the batch once per candidate configuration (blocks per
 * compute unit 2/4/all co-resident (untuned default: all), GEMM tiles per
 * task 1/2, translation column tiles per task 1/4) after a warm-up, keeps
 * the fastest and reports it in
 * choice[3] = {blocks per CU, GEMM tiles per task, translation tiles per
 * task} (may be NULL).  Writes K like occk_batch_run.  Synchronous. */
int32_t occk_batch_tune(occk_batch* plan, const double* const* C, const int64_t* ldc, double* const* K,
                        const int64_t* ldk, void* hip_stream, int32_t* choice);

/* The one-call form of a plan (the batched entry point of the hot path):
 * occk_batch_create, occk_batch_run and occk_batch_free in turn, so K[k]
 * (columns 0..nocc[k]-1, overwritten) holds K^ff of system k when it
 * returns (it synchronises the device when freeing the plan).  Arguments as
 * for occk_batch_create and occk_batch_run; the I/O arrays are checked
 * before any plan is made.  A caller that runs the same systems again keeps
 * a plan instead: this call rebuilds the tables, the operators and the
 * workspaces every time. */
int32_t occk_far_K_batched(int32_t nsys, occk_tree* const* trees, const double* const* C, const int64_t* ldc,
                           const int32_t* nocc, const occk_far_opts* opts, double* const* K, const int64_t* ldk,
                           void* hip_stream);

/* nsys and the first cap nocc values of the plan. */
int32_t occk_batch_shape(const occk_batch* plan, int32_t* nsys, int32_t* nocc, int32_t cap);

/* config[6] = {blocks per CU, GEMM tiles per task, translation tiles per
 * task, number of tasks, number of stages, resident-block limit per CU} of
 * the plan's current configuration. */
int32_t occk_batch_config(const occk_batch* plan, int32_t* config);

/* Diagnostics of the last occk_batch_run/tune launch (synchronises the
 * device): for stages s < min(cap, nstage), ms[s] = wall-clock duration of
 * stage s up to and including its grid barrier, type[s] = task type of the
 * stage (0 opgen, 1 convert, 2 half transform of all columns, 3 half
 * transform of a j batch, 4 Omega, 5 translation pass, 6 L2P, 7 mirrored
 * L2P, 8 reduce; the first system that has the stage decides).  Either
 * array may be NULL; *nstage (may be NULL) receives the stage count.
 * Before the first launch only *nstage is written.  Errors: EHANDLE,
 * EINVAL, EHIP. */
int32_t occk_batch_stage_times(occk_batch* plan, double* ms, int32_t* type, int32_t cap, int32_t* nstage);

/* Frees the plan (after a device synchronisation); NULL is accepted. */
int32_t occk_batch_free(occk_batch* plan);

/* ---- learned rank per interaction-list translation ---- */

/* The selector is an MLP (24 features -> 64 -> 64 -> 8 outputs, ReLU) that
 * predicts, for one interaction-list translation (Eq. 17b), the relative
 * truncation error e_p of keeping only l, l' <= p, as log10(e_p)/4 for
 * p = 1..8.  In OCCK_RANK_LEARNED mode every interaction-list translation of
 * occk_far_K runs at the smallest p whose prediction is <= (log10_tau -
 * margin)/4, and at lmax when none is (the fixed-rank method is the
 * fallback); upward and downward translations always use lmax.  Features
 * (index: value): 0 level/depth; 1 |R|/(h(2ws+2)); 2 rho; 3 log10 rho;
 * 4..11 log10(n_l/(n_0 h^l))/4, l = 1..8 (0 beyond lmax); 12..19 l log10(rho)/4;
 * 20 log10(n_0)/10; 21 ndim/3; 22 max_d|R_d|/(h(2ws+2)); 23 log10((n_0/|R|)/S)/4
 * with S the sum of n_0/|R| over the target box's interaction list.  Here R is
 * the box-centre displacement, h the box size of the level, rho =
 * (sqrt(ndim) h/2)/|R| and n_l the norm of the source box's order-l multipole
 * components over a column sketch of the current j batch.  Weights: flat FP32 vector
 * W1[64][24], b1[64], W2[64][64], b2[64], W3[8][64], b3[8]. */
#define OCCK_SELECTOR_NFEAT 24
#define OCCK_SELECTOR_NOUT 8
#define OCCK_SELECTOR_NPARAM 6280

/* New selector with seeded He-normal weights (zero biases), rule
 * log10_tau = -6, margin = 1. */
int32_t occk_selector_create(int32_t seed, occk_selector** out);
int32_t occk_selector_free(occk_selector* sel);
/* Host copies of the flat FP32 weights [OCCK_SELECTOR_NPARAM]. */
int32_t occk_selector_get_weights(const occk_selector* sel, float* theta);
int32_t occk_selector_set_weights(occk_selector* sel, const float* theta);
int32_t occk_selector_set_rule(occk_selector* sel, float log10_tau, float margin);

/* Training data generated by the method: runs the FP64 half transform, Omega
 * and upward passes of occk_far_K for the j batch [j0, j1) (all i), then, for
 * up to max_samples interaction-list translations drawn with the seed, the
 * features and the targets log10(max(e_p, 1e-16))/4, p = 1..8, where e_p is the
 * Frobenius norm of the difference between the rank-p and the full-rank
 * translation of the source box's multipoles, divided by the norm of the
 * target box's complete local expansion (all sources, full rank), over 64
 * sketch columns.  feat
 * [max_samples*24] and target [max_samples*8] are host arrays; *nsamples
 * receives the count.  Synchronous. */
int32_t occk_selector_collect(occk_tree* tree, const double* C, int64_t ldc, int32_t nocc, int32_t j0, int32_t j1,
                              int32_t max_samples, int32_t seed, float* feat, float* target, int32_t* nsamples,
                              void* hip_stream);

/* Adam on the mean squared error over (feat, target) host arrays of n
 * samples: epochs passes in seeded random order, minibatches of batch, step
 * size lr; FP32 forward/backward kernels on the GPU.  loss[epochs] (host, may be
 * NULL) receives each epoch's mean loss.  Synchronous. */
int32_t occk_selector_train(occk_selector* sel, const float* feat, const float* target, int32_t n, int32_t epochs,
                            int32_t batch, float lr, int32_t seed, float* loss, void* hip_stream);

/* Full-batch loss and gradient [OCCK_SELECTOR_NPARAM] at the current weights
 * (FP32 kernels; for checking the backward pass).  Synchronous. */
int32_t occk_selector_grad(occk_selector* sel, const float* feat, const float* target, int32_t n, float* loss,
                           float* grad, void* hip_stream);

/* BF16 inference on host features: outputs [n*8] and ranks [n] by the rule
 * (either may be NULL), ranks capped at lmax.  Synchronous. */
int32_t occk_selector_predict(occk_selector* sel, const float* feat, int32_t n, int32_t lmax, float* out,
                              int32_t* rank, void* hip_stream);

/* Weights file: "OCCKSEL1", int32 dims {24, 64, 8}, float {log10_tau, margin},
 * the FP32 weights, uint64 FNV-1a checksum of the weight bytes.  load rejects
 * a wrong header, checksum or non-finite weight (EINVAL / ENONFINITE) and then
 * leaves the selector unchanged. */
int32_t occk_selector_save(const occk_selector* sel, const char* path);
int32_t occk_selector_load(occk_selector* sel, const char* path);

/* Histogram hist[9] of the ranks chosen for interaction-list translations by
 * the learned calls since the previous read, one count per translation per j
 * batch (synchronises; then clears). */
int32_t occk_rank_stats(occk_tree* tree, int64_t* hist);

/* ---- per-kernel timing ---- */

/* kernel classes of one occk_far_K call */
enum {
  OCCK_K_OPGEN = 0,   /* translation operators, FP64 recurrences              */
  OCCK_K_HALF = 1,    /* H = O^B C_B[:, J]            Eq. (15a)                */
  OCCK_K_OMEGA = 2,   /* Omega = C_B^T H               Eq. (15b)                */
  OCCK_K_UP = 3,      /* all upward translation launches, Eq. (17a)            */
  OCCK_K_DOWN = 4,    /* all interaction-list + downward launches, Eq. (17b,c) */
  OCCK_K_L2P = 5,     /* per-leaf K partials, Eq. (18)                          */
  OCCK_K_REDUCE = 6,  /* sum of the per-leaf partials into K                    */
  OCCK_K_CONVERT = 7, /* operand conversion of the mixed-precision paths       */
  OCCK_K_SELECT = 8,  /* learned ranks: multipole norms, features, MLP         */
  /* single kernels inside the classes above (their time also counts there) */
  OCCK_K_HT = 9,          /* all-column half transform of the symmetric schedule, in HALF */
  OCCK_K_UP_WALK = 10,    /* upward subtree walk, in UP                               */
  OCCK_K_DOWN_WALK = 11,  /* downward subtree walk, in DOWN                           */
  OCCK_K_L2P_DIRECT = 12, /* direct L2P GEMM, in L2P                                  */
  OCCK_K_L2P_MIRROR = 13, /* mirrored L2P GEMM of the symmetric schedule, in L2P      */
  OCCK_K_TREE = 14,       /* whole tree of a column group in LDS, in DOWN             */
  OCCK_K_NCLASS = 15
};

/* While enabled, every occk_far_K on the handle records a HIP event pair on
 * its stream around each kernel class (a small serialisation cost). */
int32_t occk_profile_enable(occk_tree* tree, int32_t enable);

/* Waits for the recorded events and returns, per class, the summed elapsed
 * milliseconds ms[OCCK_K_NCLASS] and launch counts launches[OCCK_K_NCLASS]
 * (either may be NULL) since the previous read; then clears them. */
int32_t occk_profile_read(occk_tree* tree, double* ms, int64_t* launches);

/* ---- diagnostics (not needed by callers of the method) ---- */

/* Lane-layout probe of the MFMA instructions used by the kernels: multiplies a
 * one-hot 16xK A (1 at row ia, column ka) by a one-hot Kx16 B (1 at row ka,
 * column jb) on the GPU and writes every lane's four accumulator values to
 * host_out[64*4].  kind 0: FP64 16x16x4 (ka < 4), 1: FP32 16x16x4 (ka < 4),
 * 2: BF16 16x16x32 (ka < 32).  Synchronous.  EINVAL on out-of-range input. */
int32_t occk_debug_mfma_probe(int32_t kind, int32_t ia, int32_t ka, int32_t jb, double* host_out);

/* Copies a workspace buffer of the handle's last occk_far_K call to host
 * memory after a device synchronisation: which = 0 translation operators,
 * 1 half-transformed multipoles H of the last j batch (empty when the i and
 * j ranges coincide: that schedule reads each batch's H out of the
 * all-column half transform), 2 box data (Omega then Mloc; where the
 * downward pass ran as a subtree walk, the Mloc of the boxes below the walk's
 * roots and above the leaves are not written), 3 per-leaf K partials.
 * *count receives the element count; host may be NULL to query it.
 * ESTATE before the first occk_far_K. */
int32_t occk_debug_buffer(occk_tree* tree, int32_t which, double* host, int64_t* count);

#ifdef __cplusplus
}
#endif

#endif /* OCCK_H */
