// Device-side descriptor types and host launchers of the kernels.
#pragma once
#include <algorithm>

#include "common.hpp"

namespace hssmf {

// The descriptors of one launch.  Up to N of them travel in the kernel
// arguments themselves, so a small batch costs no upload; a larger one (or
// one recorded for replay) is an array in device memory that descs points
// to.
template <class D, int N>
struct DescBatch {
  const D* descs;   // device array, or nullptr: the inline copies
  D inl[N];
};

// descriptor i of a batch; the fields are uniform across the workgroup and
// are kept in scalar registers
template <class D, int N>
__device__ __forceinline__ D batch_get(const DescBatch<D, N>& b, int i) {
  D d = b.descs ? b.descs[i] : b.inl[i];
  static_assert(sizeof(D) % 4 == 0, "descriptor of whole words");
  int w[sizeof(D) / 4];
  __builtin_memcpy(w, &d, sizeof(d));
#pragma unroll
  for (int k = 0; k < (int)(sizeof(D) / 4); ++k) w[k] = __builtin_amdgcn_readfirstlane(w[k]);
  __builtin_memcpy(&d, w, sizeof(d));
  return d;
}

// host side: inline when the batch fits, else staged through the ring
template <class D, int N>
DescBatch<D, N> make_batch(const std::vector<D>& v, Stager& st, hipStream_t s) {
  DescBatch<D, N> b{};
  if (v.size() <= (size_t)N) std::copy(v.begin(), v.end(), b.inl);
  else b.descs = st.put_vec(v, s);
  return b;
}

// an array already in device memory
template <class D, int N>
DescBatch<D, N> device_batch(const D* p) {
  DescBatch<D, N> b{};
  b.descs = p;
  return b;
}

// A dense front (or any square matrix factored by the batched blocked LU):
// F is n x n column major (ld = ld); pivoting is restricted to rows [0, s).
struct LUFront {
  double* F;
  int* ipiv;     // s pivot rows (front-local row indices)
  int s, n, ld;
  int id;        // reported on a zero pivot
};

// extend-add: F[map[i], map[j]] += U[i, j] for i, j < u
struct EADesc {
  const double* U;
  double* F;
  const int* map;
  int u, ldu, ldf, pad;
};

// y[rmap ? rmap[r] : r] += alpha * sum_j M[r, j] x[xmap ? xmap[j] : j]
// (trans: M^T, i.e. r indexes columns of M)
struct GemvDesc {
  const double* M;
  const double* x;
  double* y;
  const int* xmap;
  const int* ymap;
  int rows, cols, ld, trans;
  double alpha;
  int overwrite;   // y = alpha M x instead of y += alpha M x
  int pad;
};

// triangular solve of one front's F11 block in place on a vector
struct TrsvDesc {
  const double* F;   // F11 at F, ld
  const int* ipiv;   // pivots (nullptr: none)
  double* x;         // s entries
  int s, ld;
};

// gather of the multifrontal right-hand side (forward sweep): for front
// local index i: v = (i < s ? y[sep_lo + i] : 0) + sum_c w_c[inv_c[i]];
// written to y[sep_lo + i] or w[i - s].
struct RhsDesc {
  double* y;       // global vector (new ordering)
  double* w;       // this front's update vector (u)
  const double* wc[2];
  const int* inv[2];
  int n, s, sep_lo, nkids;
};

void launch_fill(double* p, int64_t n, double v, hipStream_t s);
void launch_assemble(double* base, const int64_t* dst, const int64_t* src, const double* val,
                     int64_t count, hipStream_t s);
void launch_extend_add(const EADesc* d, int nd, int max_u, hipStream_t s);
void launch_lu_panel(const LUFront* fr, int nf, int jb, int nb, int* info, hipStream_t s, double flops = 0.0);
// the same panel as two kernels: the F11 rows resident in LDS (max_m1 = the
// largest s - jb of the batch), then the F21 rows (max_u = largest n - s)
bool lu_panel_split_fits(int max_m1, int nb);
void launch_lu_panel_split(const LUFront* fr, int nf, int jb, int nb, int max_m1, int max_u, int* info, hipStream_t s,
                           double flops = 0.0);
// interchanges p0 .. p0 + np - 1 (clamped to s) on the columns [c0, c1)
// (c1 < 0: up to n, else clamped to s), the pivot columns excepted
void launch_laswp(const LUFront* fr, int nf, int p0, int np, int c0, int c1, int max_n, hipStream_t s);
// rows [jb, jb + min(nb, s - jb)) of U12 (nb <= 64) on the columns [c0, c1)
// (c0 < 0: from the end of those rows' diagonal block; c1 < 0: up to n;
// explicit bounds clamped to s)
void launch_trsm_u12(const LUFront* fr, int nf, int jb, int nb, int c0, int c1, int max_n, hipStream_t s);
// gx: workgroups along x (ceil(rows / 16) non-transposed, ceil(cols / 4)
// transposed, the largest over the batch)
void launch_gemv(const GemvDesc* d, int nd, int gx, hipStream_t s);
// kind: 0 = L^{-1} P (unit lower, pivots first), 1 = U^{-1} (upper),
// 2 = U^{-T}, 3 = P^T L^{-T} (unit, pivots last), 4 = L^{-1} (non-unit
// lower), 5 = L^{-T} (non-unit lower, transposed)
void launch_trsv(const TrsvDesc* d, int nd, int kind, int max_s, hipStream_t s);
// The same solves with one workgroup per block of 64 entries of each system
// (identical results; an ordinary launch of nd ceil(max_s / 64) workgroups,
// also inside a graph).  trsv_multi_use: whether a batch takes it (systems of
// at least 256 entries; at most 32 systems for the untransposed kinds).  ws holds 3 + nd (ceil(max_s / 64) + 1) ints, zero
// before the first launch and kept between launches; *err != 0 after a
// launch means a bounded wait gave up and the results are invalid.
bool trsv_multi_use(int nd, int kind, int max_s);
void launch_trsv_multi(const TrsvDesc* d, int nd, int kind, int max_s, int* ws, int* err, hipStream_t s);
void launch_rhs_gather(const RhsDesc* d, int nd, int max_n, hipStream_t s);

}  // namespace hssmf

namespace hssmf {

// front-local sparse block A_i (rows and columns local to the front, only
// entries with row < s or column < s), values read through vidx from the
// CSR value array
struct SpFront {
  const int* rowptr;
  const int* col;
  const int64_t* vidx;
};

// y[i, c] = (beta ? y : 0) + sum_e A[i, col[e]] * x[col[e], c]
struct SpmmDesc {
  SpFront A;
  const double* val;
  const double* X;
  double* Y;
  int nrows, ncols, ldx, ldy;
};

// dst[i, j] (+)= src[rmap(i), cmap(j)] (or src^T when trans), i < m, j < n
struct CopyDesc {
  const void* src;
  void* dst;
  const int* rmap;
  const int* cmap;
  int m, n, lds, ldd;
  int accumulate, trans;
  double alpha;
};

// tile of one plain copy: TR rows (one per thread of a 256-thread group,
// 256 / TR column groups) by TC = 8 * 256 / TR columns, so a column segment
// of up to 2 KB is read and written as one stretch; a transposed copy uses
// 64 x 64 tiles
__host__ __device__ inline int copy_tile_rows(int m) { return m > 128 ? 256 : (m > 64 ? 128 : 64); }

using CopyBatch = DescBatch<CopyDesc, 32>;

// workgroups one copy descriptor can keep busy
inline int64_t copy_tiles(const CopyDesc& c) {
  if (c.m <= 0 || c.n <= 0) return 0;
  if (c.trans) return (int64_t)((c.m + 63) / 64) * ((c.n + 63) / 64);
  const int tr = copy_tile_rows(c.m), tc = 8 * 256 / tr;
  return (int64_t)((c.m + tr - 1) / tr) * ((c.n + tc - 1) / tc);
}

// what element extraction needs to know about a front F_i = A_i (+) U_kids
// A child's update matrix U = F22 - Theta^* Phi kept in low-rank form
// (Sec. 4.4), for entry extraction (Sec. 4.5): an entry of F22 is read from
// a leaf block D when both indices fall in one leaf, else it is row a of
// Ubig of the row side's child x of their lowest common ancestor p times
// column b of T (B12 Vbig^T or B21 Vbig^T of p, r_x x m_y, ld max(r_x, 1)).
// Ubig is kept transposed so that row a is contiguous.
struct HssKidNode {
  int lo, m;            // rows [lo, lo + m) of the update set
  int parent, depth;    // table index of the parent (-1 at the top), depth below the top
  int r;                // row rank
  int kid0;             // table index of the first child (-1 at a leaf)
  const double* D;      // leaf: m x m
  const double* UT;     // Ubig^T, r x m (ld max(r, 1))
  const double* T12;    // non-leaf: B12 Vbig_{kid1}^T
  const double* T21;    // non-leaf: B21 Vbig_{kid0}^T
};
struct HssKidDev {
  int u, mk, nnode;
  const int* leaf_of;   // u: table index of the leaf holding each row
  const HssKidNode* nodes;
  const double* ThT;    // Theta^T, mk x u
  const double* Phi;    // mk x u
};

struct FrontOpDev {
  SpFront A;
  const double* val;
  const double* U[2];
  const HssKidDev* hk[2];   // a child in low-rank form (U null), else null
  const int* inv[2];   // front-local index -> child-local index or -1
  int ldu[2];
  int nkids, n;
};

struct ExtractDesc {
  double* dst;
  const int* I;
  const int* J;
  int m, n, ldd, fop;
};


struct TrsmDesc {
  const double* T;
  double* X;
  int n, ncols, ldt, ldx;
  int b0, bs;
};
using TrsmBatch = DescBatch<TrsmDesc, 48>;

void launch_rng(double* R, int ldr, const int* orig, int nrows, int c0, int nc, uint64_t seed, hipStream_t s);
void launch_spmm(const SpmmDesc* d, int nd, int max_rows, int max_cols, hipStream_t s);
// max_tiles: largest copy_tiles() over the descriptors
void launch_copy(const CopyBatch& d, int nd, int64_t max_tiles, int f32, hipStream_t s);
// entries of the fronts' operators: A_i and dense children's update
// matrices in one pass (one thread per entry), then, when lowrank is set,
// the low-rank children's entries added by a second pass (one wavefront per
// entry)
void launch_extract(const ExtractDesc* d, int nd, const FrontOpDev* fops, int64_t max_elems, bool lowrank,
                    hipStream_t s);
// dst (m x k, ld ldd) = Pi [I; E]: dst[perm[i], :] = row i of [I; E]
struct InterpDesc {
  double* dst;
  const int* perm;
  const double* E;   // (m-k) x k, ld m-k
  int m, k, ldd, pad;
};
void launch_interp_dense(const InterpDesc* d, int nd, int64_t max_elems, hipStream_t s);
// row interchanges ipiv[0..k) (reverse: undone) on all ncols columns of M;
// perm_ws: k ints of device workspace
void launch_pivots(double* M, int ld, int ncols, const int* ipiv, int k, int reverse, int* perm_ws, hipStream_t s);
// logical T(i,j) = trans ? T[j + i ld] : T[i + j ld]; solve rows [b0, b0+bs) in place
void launch_trsm_block(const TrsmBatch& d, int nd, int lower, int unit, int trans, int max_cols, hipStream_t s);
void launch_convert(const double* src, void* dst, int64_t n, int to_bf16, hipStream_t s);
// round x to the low precision in place and write the low-precision copy
void launch_round_lp(double* x, void* lp, int64_t n, int to_bf16, hipStream_t s);

}  // namespace hssmf

namespace hssmf {

// Column-pivoted QR for the interpolative decomposition, spread over several
// workgroups per problem with one launch per pivot step (see k_id.hip).
struct IDProb {
  const double* S;      // m x d samples (rows are the candidates), ld lds
  double* W;            // d x m work, ld d
  double* norms;        // m
  double* alpha;        // min(m, d): R diagonal
  double* slots;        // exchange records between a problem's workgroups (layout per kernel)
  double* R1;           // k x k scratch (upper triangle, pivot order)
  double* W2;           // k x (m - k) scratch: R2, then X = R1^{-1} R2
  int* perm;            // output: position -> candidate
  int* ipos;            // candidate -> position
  int* state;           // [0] done, [1] rank
  double* first;        // first pivot norm
  unsigned char* active;
  double* cand;         // per step buffer x P x d: each workgroup's best candidate column (layout per kernel)
  int* hdone;           // null, or a flag in mapped host memory that the stop step sets (stepwise path)
  const int* force;     // null, or (resident kernel) the pivot order to take: kf candidates
  int m, d, lds, P;     // P workgroups of kIDCols candidates each
  int wg0, kf;          // first workgroup of this problem in the launch grid; length of force
  double eps;           // relative stopping tolerance (Sec. 5.3)
  double atol;          // absolute stopping tolerance (0: the relative rule alone)
};
constexpr int kIDCols = 8;

void launch_id_init(const IDProb* p, int np, int total_wg, int max_d, hipStream_t s);
// wgmap[w] = (problem, workgroup within the problem) of grid workgroup w
void launch_id_step(const IDProb* p, const int2* wgmap, int total_wg, int t, int max_d, hipStream_t s);
void launch_id_finish(const IDProb* p, int np, int max_m, hipStream_t s);
// Strong-RRQR interchange test of the problems idx[0..n) (Gu and Eisenstat,
// rank k = state[1] fixed), after launch_id_finish and before any solve:
//  - launch_srrqr_eye writes the k x k identity into columns [m-k, m) of
//    W2 (k x m, ld k; columns [0, m-k) hold R2), so that one upper
//    triangular solve with R1 leaves X = R1^{-1} R2 and Z = R1^{-1} there;
//  - launch_srrqr_test then finds, per problem, the largest
//    rho_ij = X_ij^2 + gamma_j^2 sum_l Z_il^2 over e = i + k j (ties to the
//    lowest e), gamma_j the 2-norm of rows k.. of remaining column j in W:
//    rho[x] and e[x] for problem idx[x].  max_m bounds every problem's m.
void launch_srrqr_eye(const IDProb* p, const int* idx, int n, int max_k, hipStream_t s);
void launch_srrqr_test(const IDProb* p, const int* idx, int n, int max_m, double* rho, int* e, hipStream_t s);

// Copy (HBM GB/s), FP64 FMA loop and FP64 matrix-core loop (TFLOP/s) rates.
void measure_peaks(hipStream_t s, double* hbm_gbps, double* valu_tflops, double* mfma_tflops);
// Cooperative variant: every pivot step of the listed problems in one launch
// whose workgroups are all resident (hipLaunchCooperativeKernel), with the
// candidates kept in registers and a per-problem barrier between steps.
// id_coop_capacity(max_d) = workgroups that can be resident at once (0 when
// the device has no cooperative launch or max_d > 1024).  slots are then
// 2 x P x 4 doubles with every step tag (entry 2) preset to -1, and *err
// zero before the launch; *err != 0 afterwards means a wait gave up and the
// results are invalid.
int id_coop_capacity(int max_d);
void launch_id_coop(const IDProb* p, const int2* wgmap, int total_wg, int max_d, int* err, hipStream_t s);

// Resident variant (k_idres.hip): every pivot step in one launch, the
// candidates of a problem resident in the registers of P workgroups of
// id_res_candidates(max_d, max_m) candidates each, for the template the
// launch's largest sample count and largest problem select (0: max_d above
// 640, or max_m above twice the rows the template holds).  Problems with
// P = 1 need no other workgroup; a launch holding any problem with P > 1
// must be cooperative (coop = true, at most id_res_capacity(max_d, max_m)
// workgroups), with that problem's slots (3 x P x 2 doubles, all NaN) and
// cand (3 x P x d) set and *err zero; *err != 0
// afterwards means a wait gave up and the results are invalid.  Every
// launch of one pass must take the same (max_d, max_m).  A launch with
// forced = true (its own instantiations; every problem it covers has force
// set) takes the candidates force[0..kf) as each problem's pivots, in that order
// (kf <= min(m, d), distinct), and stops after them: its rank is kf, and
// its pivot order, R diagonal and W are those of a Householder QR in that
// order with the same interchange bookkeeping.
int id_res_candidates(int max_d, int max_m);
int id_res_capacity(int max_d, int max_m);
void launch_id_res(const IDProb* p, const int2* wgmap, int total_wg, int max_d, int max_m, bool coop, int* err,
                   hipStream_t s);
// The same kernel with one template per problem: id_res_template(d, m) is
// the template a problem of d samples and m rows takes on its own (-1: none
// holds it), id_res_template_candidates / _capacity that template's
// candidates per workgroup and cooperative capacity.  A problem's P then
// follows from its own template, and every launch that covers it must use
// that template.
int id_res_template(int d, int m);
int id_res_template_candidates(int tpl);
int id_res_template_capacity(int tpl);
void launch_id_res_template(int tpl, const IDProb* p, const int2* wgmap, int total_wg, bool coop, int* err,
                            hipStream_t s, bool forced = false);

}  // namespace hssmf

namespace hssmf {

// one 32-column panel of a blocked Householder QR of C[:, 0:ncols_qr]
// (column major, m rows, ld m): factors columns [j0, j0+nb) in place (R on
// and above the diagonal), writes the reflectors as a dense m x nb block Y
// (zeros above row j0+l in column l) and the nb x nb upper triangular T of
// the compact WY form  H_j0 ... H_j0+nb-1 = I - Y T Y^T
struct PanelDesc {
  double* C;
  double* Y;
  double* T;
  int m, j0, nb, pad;
};
constexpr int kPanel = 32;
// max_mp: the largest m - j0 of the batch (rows of a panel)
void launch_qr_panel(const PanelDesc* d, int nd, int max_mp, hipStream_t s);

}  // namespace hssmf
