// Numeric multifrontal factorization on the GPU (Sec. 3.2 and Sec. 4).
//
// Fronts are processed by elimination-tree height, all fronts of one height
// together.  Dense fronts: zero fill, assembly of original entries,
// extend-add of the children's update matrices (one launch per child slot),
// batched blocked partial LU.  HSS fronts: keyed random matrix, samples
// F R and F^T R by skinny extend-add (sparse product plus GEMMs with the
// children's update matrices through row maps), Alg. 1 bottom-up over the
// HSS levels with the adaptive-rank loop, ULV-like factorization of F11,
// the low-rank Schur product Theta^* Phi and the update matrix
// F22 - Theta^* Phi for the parent.  Only ranks and pivot orders of the IDs
// come back to the host (one synchronization per HSS level).
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <limits>
#include <map>
#include <numeric>

#include "solver.hpp"

namespace hssmf {

GemmType Handle::gt() const {
  return o.gemm_prec == HSSMF_PREC_FP32 ? GEMM_F32_D : o.gemm_prec == HSSMF_PREC_BF16 ? GEMM_BF16_D : GEMM_F64;
}

namespace {

GemmDesc G(const void* A, int lda, int tA, const void* B, int ldb, int tB, void* C, int ldc, int m, int n, int k,
           double al, double be, const int* bmap = nullptr, const int* cmap = nullptr, const int* amap = nullptr) {
  GemmDesc g{};
  g.A = A; g.B = B; g.C = C;
  g.lda = lda; g.ldb = ldb; g.ldc = ldc;
  g.transA = tA; g.transB = tB;
  g.m = m; g.n = n; g.k = k;
  g.alpha = al; g.beta = be;
  g.amap = amap; g.bmap = bmap; g.cmap = cmap;
  return g;
}

CopyDesc Cp(const void* src, int lds, const int* rmap, void* dst, int ldd, int m, int n, int acc = 0,
            double alpha = 1.0, const int* cmap = nullptr, int trans = 0) {
  CopyDesc c{};
  c.src = src; c.dst = dst; c.rmap = rmap; c.cmap = cmap;
  c.m = m; c.n = n; c.lds = lds; c.ldd = ldd;
  c.accumulate = acc; c.trans = trans; c.alpha = alpha;
  return c;
}

void run_gemm(Handle& h, const std::vector<GemmDesc>& v, GemmType t = GEMM_F64) {
  if (!v.empty()) gemm_batched(v, t, h.stager, h.st, h.o.gemm_tile);
}

void run_copy(Handle& h, const std::vector<CopyDesc>& v) {
  std::vector<CopyDesc> w;
  int64_t mx = 0;
  for (auto& c : v)
    if (c.m > 0 && c.n > 0) { w.push_back(c); mx = std::max<int64_t>(mx, copy_tiles(c)); }
  if (w.empty()) return;
  launch_copy(make_batch<CopyDesc, 32>(w, h.stager, h.st), (int)w.size(), mx, 0, h.st);
}

void run_extract(Handle& h, const std::vector<ExtractDesc>& v, const FrontOpDev* fops) {
  std::vector<ExtractDesc> w;
  int64_t mx = 0;
  for (auto& c : v)
    if (c.m > 0 && c.n > 0) { w.push_back(c); mx = std::max<int64_t>(mx, (int64_t)c.m * c.n); }
  if (w.empty()) return;
  launch_extract(h.stager.put_vec(w, h.st), (int)w.size(), fops, mx, h.o.hss_update == HSSMF_UPDATE_LOWRANK, h.st);
}

void run_interp(Handle& h, const std::vector<InterpDesc>& v) {
  std::vector<InterpDesc> w;
  int64_t mx = 0;
  for (auto& c : v)
    if (c.m > 0 && c.k > 0) { w.push_back(c); mx = std::max<int64_t>(mx, (int64_t)c.m * c.k); }
  if (w.empty()) return;
  launch_interp_dense(h.stager.put_vec(w, h.st), (int)w.size(), mx, h.st);
}

}  // namespace

// ------------------------------------------------------- blocked LU -------
// Partial LU of a batch of fronts (pivoting inside F11).  Block columns of
// KB = 128 are factored panel by panel (NB = 32 wide: panel kernel, then
// the interchanges, the U12 rows and the update restricted to the block
// column); the block's interchanges then go to the columns outside it, its
// U12 rows are solved against the 128 x 128 unit-lower diagonal block (two
// 64-row halves), and the trailing matrix takes one update with k = 128.
// This is the usual two-level blocking of a right-looking LU: the trailing
// matrix is read and written once per 128 columns instead of once per 32.
constexpr int NB = 32;
constexpr int KB = 128;

void blocked_lu(Handle& h, const std::vector<LUFront>& fronts) {
  if (fronts.empty()) return;
  LUFront* d = upload(h, fronts);
  int maxs = 0, maxn = 0;
  for (auto& f : fronts) { maxs = std::max(maxs, f.s); maxn = std::max(maxn, f.n); }
  const int nf = (int)fronts.size();
  for (int jb = 0; jb < maxs; jb += KB) {
    // the block column, panel by panel
    for (int jp = jb; jp < std::min(jb + KB, maxs); jp += NB) {
      double pfl = 0.0;   // panel flops: w columns of height m = n - jp, m w^2 - w^3 / 3
      if (prof::enabled())
        for (auto& f : fronts)
          if (jp < f.s) {
            const double w = std::min(NB, f.s - jp), m = f.n - jp;
            pfl += m * w * w - w * w * w / 3.0;
          }
      int m1 = 0, mu = 0;
      for (auto& f : fronts)
        if (jp < f.s) { m1 = std::max(m1, f.s - jp); mu = std::max(mu, f.n - f.s); }
      if (lu_panel_split_fits(m1, NB)) launch_lu_panel_split(d, nf, jp, NB, m1, mu, h.d_info, h.st, pfl);
      else launch_lu_panel(d, nf, jp, NB, h.d_info, h.st, pfl);
      launch_laswp(d, nf, jp, NB, jb, jb + KB, maxn, h.st);
      launch_trsm_u12(d, nf, jp, NB, -1, jb + KB, maxn, h.st);
      std::vector<GemmDesc> g;
      for (auto& f : fronts) {
        if (jp >= f.s) continue;
        const int w = std::min(NB, f.s - jp);
        const int nc = std::min(jb + KB, f.s) - (jp + w);
        const int m2 = f.n - jp - w;
        if (nc <= 0 || m2 <= 0) continue;
        const int64_t ld = f.ld;
        g.push_back(G(f.F + (jp + w) + jp * ld, f.ld, 0, f.F + jp + (jp + w) * ld, f.ld, 0,
                      f.F + (jp + w) + (jp + w) * ld, f.ld, m2, nc, w, -1.0, 1.0));
      }
      run_gemm(h, g);
    }
    // the block's interchanges on the columns outside it
    launch_laswp(d, nf, jb, KB, 0, -1, maxn, h.st);
    // its U12 rows against the unit-lower diagonal block, 64 rows at a time
    launch_trsm_u12(d, nf, jb, 64, jb + KB, -1, maxn, h.st);
    std::vector<GemmDesc> g;
    for (auto& f : fronts) {
      if (jb >= f.s) continue;
      const int kb = std::min(KB, f.s - jb), nc = f.n - jb - kb;
      if (kb <= 64 || nc <= 0) continue;
      const int64_t ld = f.ld;
      g.push_back(G(f.F + (jb + 64) + jb * ld, f.ld, 0, f.F + jb + (jb + kb) * ld, f.ld, 0,
                    f.F + (jb + 64) + (jb + kb) * ld, f.ld, kb - 64, nc, 64, -1.0, 1.0));
    }
    run_gemm(h, g);
    launch_trsm_u12(d, nf, jb + 64, 64, jb + KB, -1, maxn, h.st);
    // the trailing update, k = the block width
    g.clear();
    for (auto& f : fronts) {
      if (jb >= f.s) continue;
      const int kb = std::min(KB, f.s - jb), m2 = f.n - jb - kb;
      if (m2 <= 0) continue;
      const int64_t ld = f.ld;
      g.push_back(G(f.F + (jb + kb) + jb * ld, f.ld, 0, f.F + jb + (jb + kb) * ld, f.ld, 0,
                    f.F + (jb + kb) + (jb + kb) * ld, f.ld, m2, m2, kb, -1.0, 1.0));
    }
    run_gemm(h, g);
  }
}

// X := op(T)^{-1} X for a triangular T (n x n), X n x ncols; blocks of 64
// solved by trsm_block, off-diagonal blocks applied with GEMMs
void tri_solve_many(Handle& h, const double* T, int ldt, int n, double* X, int ldx, int ncols, bool lower,
                    bool unit, bool trans) {
  if (n <= 0 || ncols <= 0) return;
  auto run_block = [&](int b0, int bs) {
    TrsmBatch tb{};
    tb.inl[0] = TrsmDesc{T, X, n, ncols, ldt, ldx, b0, bs};
    launch_trsm_block(tb, 1, lower, unit, trans, ncols, h.st);
  };
  // logical T(i,j) = trans ? T[j,i] : T[i,j]; the block (rows R, cols C)
  // of the logical matrix as a GEMM operand
  auto blk = [&](int r0, int c0) -> const double* {
    return trans ? T + c0 + (int64_t)r0 * ldt : T + r0 + (int64_t)c0 * ldt;
  };
  if (lower) {
    for (int b0 = 0; b0 < n; b0 += 64) {
      int bs = std::min(64, n - b0);
      run_block(b0, bs);
      int rest = n - b0 - bs;
      if (rest > 0)
        run_gemm(h, {G(blk(b0 + bs, b0), ldt, trans, X + b0, ldx, 0, X + b0 + bs, ldx, rest, ncols, bs, -1.0, 1.0)});
    }
  } else {
    for (int b1 = n; b1 > 0; b1 -= 64) {
      int b0 = std::max(0, b1 - 64), bs = b1 - b0;
      run_block(b0, bs);
      if (b0 > 0) run_gemm(h, {G(blk(0, b0), ldt, trans, X + b0, ldx, 0, X, ldx, b0, ncols, bs, -1.0, 1.0)});
    }
  }
}

// X := T^{-1} X for a batch of upper triangular T (non-unit), blocks of 64
// from the bottom, all problems of the batch in the same launches
void tri_solve_upper_batched(Handle& h, const std::vector<TriProb>& ps) {
  int nmax = 0, cmax = 0;
  for (auto& p : ps) { nmax = std::max(nmax, p.n); cmax = std::max(cmax, p.ncols); }
  for (int j = 0; 64 * j < nmax; ++j) {
    std::vector<TrsmDesc> td;
    std::vector<GemmDesc> g;
    for (auto& p : ps) {
      const int b1 = p.n - 64 * j;
      if (b1 <= 0) continue;
      const int b0 = std::max(0, b1 - 64), bs = b1 - b0;
      td.push_back({p.T, p.X, p.n, p.ncols, p.ldt, p.ldx, b0, bs});
      if (b0 > 0)
        g.push_back(G(p.T + (int64_t)b0 * p.ldt, p.ldt, 0, p.X + b0, p.ldx, 0, p.X, p.ldx, b0, p.ncols, bs, -1.0, 1.0));
    }
    if (td.empty()) continue;
    launch_trsm_block(make_batch<TrsmDesc, 48>(td, h.stager, h.st), (int)td.size(), 0, 0, 0, cmax, h.st);
    run_gemm(h, g);
  }
}

// ------------------------------------------------------------ HSS ---------
namespace {

struct NRef {
  HFront* F;
  int t;
  HNode& n() const { return F->nd[t]; }
};

// interchanges per ID at most in the strong rank-revealing QR
constexpr int kSrrqrMaxSwaps = 64;

double* dalloc(Handle& h, int64_t n) { return h.cur->get<double>((size_t)std::max<int64_t>(n, 1)); }
int* ialloc(Handle& h, int64_t n) { return h.cur->get<int>((size_t)std::max<int64_t>(n, 1)); }
// temporaries: every launch that uses them is ordered on the one stream
// before any later reuse of the memory, so the arenas can be recycled
// without waiting
double* salloc(Handle& h, int64_t n) { return h.sarena.get<double>((size_t)std::max<int64_t>(n, 1)); }
int* sialloc(Handle& h, int64_t n) { return h.sarena.get<int>((size_t)std::max<int64_t>(n, 1)); }
double* lalloc(Handle& h, int64_t n) { return h.larena.get<double>((size_t)std::max<int64_t>(n, 1)); }

// allocate / grow R, S^r, S^c of a front to hold dnew columns
void grow_samples(Handle& h, HFront& F, int dnew) {
  if (dnew <= F.dcap) return;
  // geometric growth keeps the copies of every growth round within 2x
  int cap = std::max(dnew, std::min(2 * F.dcap, h.o.d_max));
  double* R = lalloc(h, (int64_t)F.n * cap);
  double* Sr = lalloc(h, (int64_t)F.n * cap);
  double* Sc = lalloc(h, (int64_t)F.n * cap);
  if (F.R && F.d > 0) {
    size_t bytes = sizeof(double) * (size_t)F.n * F.d;
    HIP_CHECK(hipMemcpyAsync(R, F.R, bytes, hipMemcpyDeviceToDevice, h.st));
    HIP_CHECK(hipMemcpyAsync(Sr, F.Sr, bytes, hipMemcpyDeviceToDevice, h.st));
    HIP_CHECK(hipMemcpyAsync(Sc, F.Sc, bytes, hipMemcpyDeviceToDevice, h.st));
  }
  if (h.o.gemm_prec != HSSMF_PREC_FP64) {
    const size_t eb = h.o.gemm_prec == HSSMF_PREC_BF16 ? 2 : 4;
    void* lp = h.larena.alloc(eb * (size_t)F.n * cap);
    if (F.Rlp && F.d > 0)
      HIP_CHECK(hipMemcpyAsync(lp, F.Rlp, eb * (size_t)F.n * F.d, hipMemcpyDeviceToDevice, h.st));
    F.Rlp = lp;
  }
  F.R = R; F.Sr = Sr; F.Sc = Sc;
  if (h.o.power_q > 0) {
    // R^r and R^c of the power iteration, grown alike
    double* Rr = lalloc(h, (int64_t)F.n * cap);
    double* Rc = lalloc(h, (int64_t)F.n * cap);
    if (F.Rr && F.d > 0) {
      size_t bytes = sizeof(double) * (size_t)F.n * F.d;
      HIP_CHECK(hipMemcpyAsync(Rr, F.Rr, bytes, hipMemcpyDeviceToDevice, h.st));
      HIP_CHECK(hipMemcpyAsync(Rc, F.Rc, bytes, hipMemcpyDeviceToDevice, h.st));
    }
    F.Rr = Rr;
    F.Rc = Rc;
  }
  F.dcap = cap;
}

// new columns of R: keyed Gaussian generator, then (mixed precision) one
// rounding to the product precision, kept in both copies so every use of R
// sees the same rounded values
void gen_random(Handle& h, HFront& F, int c0, int nc) {
  launch_rng(F.R, F.n, F.orig, F.n, c0, nc, h.o.seed, h.st);
  if (h.o.gemm_prec != HSSMF_PREC_FP64) {
    const int bf = h.o.gemm_prec == HSSMF_PREC_BF16;
    char* lp = static_cast<char*>(F.Rlp) + (size_t)c0 * F.n * (bf ? 2 : 4);
    launch_round_lp(F.R + (int64_t)c0 * F.n, lp, (int64_t)F.n * nc, bf, h.st);
  }
}

// A child whose update matrix U = F22 - Theta^* Phi is kept in low-rank
// form, sampled for its parent (Sec. 4.4): U X = F22 X - Theta^* (Phi X)
// and U^T X = F22^T X - Phi^T (Theta X) with X = R(map, cols), F22 X by
// the HSS matrix-vector product of the q-subtree: up-sweep through the
// interpolative generators (V^T X, level by level from the leaves), the
// sibling couplings B12, B21, down-sweep through U from the top, the leaf
// blocks D; F22^T X likewise with U and V exchanged, B transposed and D^T.
// Every product is a batched FP64 GEMM over all jobs; the leaf terms go
// straight into the parent's samples through the child-to-parent row map.
struct LrJob {
  HFront* F;        // the parent
  HFront* C;        // the child in low-rank form
  const int* map;   // child update index -> parent local row (device)
  int64_t off;      // first sample column times F->n
};

void sample_lowrank(Handle& h, const std::vector<LrJob>& jobs, int nc) {
  if (jobs.empty() || nc <= 0) return;
  // per non-leaf node of each q-subtree: stacked children's up-sweep
  // results (XS: V^T side, mc rows; XT: U^T side, mr rows) and down-sweep
  // inputs (YS: mr rows; YT: mc rows)
  struct Buf {
    double *XS = nullptr, *YS = nullptr, *XT = nullptr, *YT = nullptr;
  };
  std::vector<std::vector<Buf>> bufs(jobs.size());
  int maxh = 0;
  for (size_t j = 0; j < jobs.size(); ++j) {
    HFront& C = *jobs[j].C;
    bufs[j].assign(C.nd.size(), Buf{});
    for (int t = 0; t < (int)C.nd.size(); ++t) {
      const HNode& nd = C.nd[t];
      if (t == C.root || nd.lo < C.s || nd.leaf()) continue;
      Buf& b = bufs[j][t];
      b.XS = salloc(h, (int64_t)std::max(nd.mc, 1) * nc);
      b.YT = salloc(h, (int64_t)std::max(nd.mc, 1) * nc);
      b.XT = salloc(h, (int64_t)std::max(nd.mr, 1) * nc);
      b.YS = salloc(h, (int64_t)std::max(nd.mr, 1) * nc);
    }
    maxh = std::max(maxh, C.nd[C.q].height);
  }
  auto in_q = [](const HFront& C, int t) { return t != C.root && C.nd[t].lo >= C.s; };
  // offsets of a node's blocks in its parent's stacked buffers
  auto offs = [](const HFront& C, int t, int& oc, int& orr) {
    const HNode& p = C.nd[C.nd[t].parent];
    const bool first = p.kid[0] == t;
    oc = first ? 0 : C.nd[p.kid[0]].c;
    orr = first ? 0 : C.nd[p.kid[0]].r;
  };
  // up-sweep
  for (int hh = 0; hh < maxh; ++hh) {
    std::vector<GemmDesc> g;
    for (size_t j = 0; j < jobs.size(); ++j) {
      const LrJob& jb = jobs[j];
      HFront& F = *jb.F;
      HFront& C = *jb.C;
      for (int t = 0; t < (int)C.nd.size(); ++t) {
        const HNode& nd = C.nd[t];
        if (!in_q(C, t) || t == C.q || nd.height != hh) continue;
        const Buf& pb = bufs[j][nd.parent];
        const HNode& p = C.nd[nd.parent];
        int oc, orr;
        offs(C, t, oc, orr);
        if (nd.leaf()) {
          const int* bm = jb.map + (nd.lo - C.s);
          const double* X = F.R + jb.off;
          g.push_back(G(nd.Vd, nd.m(), 1, X, F.n, 0, pb.XS + oc, p.mc, nd.c, nc, nd.m(), 1.0, 0.0, bm));
          g.push_back(G(nd.Ud, nd.m(), 1, X, F.n, 0, pb.XT + orr, p.mr, nd.r, nc, nd.m(), 1.0, 0.0, bm));
        } else {
          const Buf& b = bufs[j][t];
          g.push_back(G(nd.Vd, nd.mc, 1, b.XS, nd.mc, 0, pb.XS + oc, p.mc, nd.c, nc, nd.mc, 1.0, 0.0));
          g.push_back(G(nd.Ud, nd.mr, 1, b.XT, nd.mr, 0, pb.XT + orr, p.mr, nd.r, nc, nd.mr, 1.0, 0.0));
        }
      }
    }
    run_gemm(h, g);
  }
  // sibling couplings at every non-leaf node
  {
    std::vector<GemmDesc> g;
    for (size_t j = 0; j < jobs.size(); ++j) {
      HFront& C = *jobs[j].C;
      for (int t = 0; t < (int)C.nd.size(); ++t) {
        const HNode& nd = C.nd[t];
        if (!in_q(C, t) || nd.leaf()) continue;
        const Buf& b = bufs[j][t];
        const HNode& a = C.nd[nd.kid[0]];
        const HNode& e = C.nd[nd.kid[1]];
        const int l12 = std::max(a.r, 1), l21 = std::max(e.r, 1);
        g.push_back(G(nd.B12, l12, 0, b.XS + a.c, nd.mc, 0, b.YS, nd.mr, a.r, nc, e.c, 1.0, 0.0));
        g.push_back(G(nd.B21, l21, 0, b.XS, nd.mc, 0, b.YS + a.r, nd.mr, e.r, nc, a.c, 1.0, 0.0));
        g.push_back(G(nd.B21, l21, 1, b.XT + a.r, nd.mr, 0, b.YT, nd.mc, a.c, nc, e.r, 1.0, 0.0));
        g.push_back(G(nd.B12, l12, 1, b.XT, nd.mr, 0, b.YT + a.c, nd.mc, e.c, nc, a.r, 1.0, 0.0));
      }
    }
    run_gemm(h, g);
  }
  // down-sweep through the non-leaf nodes below q, parents first
  for (int hh = maxh - 1; hh >= 1; --hh) {
    std::vector<GemmDesc> g;
    for (size_t j = 0; j < jobs.size(); ++j) {
      HFront& C = *jobs[j].C;
      for (int t = 0; t < (int)C.nd.size(); ++t) {
        const HNode& nd = C.nd[t];
        if (!in_q(C, t) || t == C.q || nd.leaf() || nd.height != hh) continue;
        const Buf& b = bufs[j][t];
        const Buf& pb = bufs[j][nd.parent];
        const HNode& p = C.nd[nd.parent];
        int oc, orr;
        offs(C, t, oc, orr);
        g.push_back(G(nd.Ud, nd.mr, 0, pb.YS + orr, p.mr, 0, b.YS, nd.mr, nd.mr, nc, nd.r, 1.0, 1.0));
        g.push_back(G(nd.Vd, nd.mc, 0, pb.YT + oc, p.mc, 0, b.YT, nd.mc, nd.mc, nc, nd.c, 1.0, 1.0));
      }
    }
    run_gemm(h, g);
  }
  // leaves: D X (D^T X), then U Y (V Y), into the parent's samples
  for (int part = 0; part < 2; ++part) {
    std::vector<GemmDesc> g;
    for (size_t j = 0; j < jobs.size(); ++j) {
      const LrJob& jb = jobs[j];
      HFront& F = *jb.F;
      HFront& C = *jb.C;
      for (int t = 0; t < (int)C.nd.size(); ++t) {
        const HNode& nd = C.nd[t];
        if (!in_q(C, t) || !nd.leaf()) continue;
        const int* rm = jb.map + (nd.lo - C.s);
        const int m = nd.m();
        if (part == 0) {
          g.push_back(G(nd.D, m, 0, F.R + jb.off, F.n, 0, F.Sr + jb.off, F.n, m, nc, m, 1.0, 1.0, rm, rm));
          g.push_back(G(nd.D, m, 1, F.R + jb.off, F.n, 0, F.Sc + jb.off, F.n, m, nc, m, 1.0, 1.0, rm, rm));
        } else if (t != C.q) {
          const Buf& pb = bufs[j][nd.parent];
          const HNode& p = C.nd[nd.parent];
          int oc, orr;
          offs(C, t, oc, orr);
          g.push_back(G(nd.Ud, m, 0, pb.YS + orr, p.mr, 0, F.Sr + jb.off, F.n, m, nc, nd.r, 1.0, 1.0, nullptr, rm));
          g.push_back(G(nd.Vd, m, 0, pb.YT + oc, p.mc, 0, F.Sc + jb.off, F.n, m, nc, nd.c, 1.0, 1.0, nullptr, rm));
        }
      }
    }
    run_gemm(h, g);
  }
  // the low-rank Schur term
  std::vector<GemmDesc> g1, g2;
  for (const LrJob& jb : jobs) {
    HFront& F = *jb.F;
    HFront& C = *jb.C;
    if (C.mk == 0) continue;
    double* T1 = salloc(h, (int64_t)C.mk * nc);
    double* T2 = salloc(h, (int64_t)C.mk * nc);
    g1.push_back(G(C.Phi, C.mk, 0, F.R + jb.off, F.n, 0, T1, C.mk, C.mk, nc, C.u, 1.0, 0.0, jb.map));
    g1.push_back(G(C.ThT, C.mk, 0, F.R + jb.off, F.n, 0, T2, C.mk, C.mk, nc, C.u, 1.0, 0.0, jb.map));
    g2.push_back(G(C.ThT, C.mk, 1, T1, C.mk, 0, F.Sr + jb.off, F.n, C.u, nc, C.mk, -1.0, 1.0, nullptr, jb.map));
    g2.push_back(G(C.Phi, C.mk, 1, T2, C.mk, 0, F.Sc + jb.off, F.n, C.u, nc, C.mk, -1.0, 1.0, nullptr, jb.map));
  }
  run_gemm(h, g1);
  run_gemm(h, g2);
}

// columns [c0, c0+nc) of S^r = F R and S^c = F^T R (Eq. FtimesR): the
// original entries by a sparse product, each child's update matrix by one
// GEMM whose B rows and C rows go through the child-to-parent map
void sample(Handle& h, const std::vector<HFront*>& fs, const std::vector<int>& c0, int nc) {
  std::vector<SpmmDesc> sp;
  int maxr = 0;
  for (size_t i = 0; i < fs.size(); ++i) {
    HFront& F = *fs[i];
    const int64_t off = (int64_t)c0[i] * F.n;
    sp.push_back({{F.a_row, F.a_col, F.a_vidx}, h.d_val, F.R + off, F.Sr + off, F.n, nc, F.n, F.n});
    sp.push_back({{F.at_row, F.at_col, F.at_vidx}, h.d_val, F.R + off, F.Sc + off, F.n, nc, F.n, F.n});
    maxr = std::max(maxr, F.n);
  }
  launch_spmm(h.stager.put_vec(sp, h.st), (int)sp.size(), maxr, nc, h.st);
  for (int slot = 0; slot < 2; ++slot) {
    std::vector<GemmDesc> g;
    std::vector<LrJob> lr;
    for (size_t i = 0; i < fs.size(); ++i) {
      HFront& F = *fs[i];
      const FrontPlan& fp = h.P.fr[F.f];
      if ((int)fp.kids.size() <= slot) continue;
      int c = fp.kids[slot];
      const FrontRT& K = h.fr[c];
      int u = h.P.fr[c].u;
      if (u == 0) continue;
      const int* map = h.fr[F.f].d_kidmap[slot];
      const int64_t off = (int64_t)c0[i] * F.n;
      if (K.hidx >= 0 && h.hf[K.hidx].lowrank) {
        lr.push_back({&F, &h.hf[K.hidx], map, off});
      } else if (h.o.gemm_prec == HSSMF_PREC_FP64) {
        g.push_back(G(K.U, K.ldu, 0, F.R + off, F.n, 0, F.Sr + off, F.n, u, nc, u, 1.0, 1.0, map, map));
        g.push_back(G(K.U, K.ldu, 1, F.R + off, F.n, 0, F.Sc + off, F.n, u, nc, u, 1.0, 1.0, map, map));
      } else {
        // low-precision products with FP32 accumulation, added into FP64 samples
        const size_t eb = h.o.gemm_prec == HSSMF_PREC_BF16 ? 2 : 4;
        const void* Rl = static_cast<const char*>(F.Rlp) + off * eb;
        g.push_back(G(K.Ulp, u, 0, Rl, F.n, 0, F.Sr + off, F.n, u, nc, u, 1.0, 1.0, map, map));
        g.push_back(G(K.Ulp, u, 1, Rl, F.n, 0, F.Sc + off, F.n, u, nc, u, 1.0, 1.0, map, map));
      }
    }
    run_gemm(h, g, h.gt());
    sample_lowrank(h, lr, nc);
  }
}

// Power iteration on columns [c0, c0+nc) (Sec. 2.2, the variant the paper
// describes as an option), once sample() has formed S^r = F R and
// S^c = F^T R there: q steps of R^r <- F^T S^r, R^c <- F S^c,
// S^r <- F R^r, S^c <- F^T R^c.  Each product is a sample() pass with its
// input and output arrays pointed elsewhere (every array n x columns, ld n);
// the half of a pass that is not wanted goes to a scratch block.  Alg. 1
// then takes R^r on the row side and R^c on the column side.
void power_iterate(Handle& h, const std::vector<HFront*>& fs, const std::vector<int>& c0, int nc) {
  const int q = h.o.power_q;
  if (q <= 0 || fs.empty() || nc <= 0) return;
  const size_t nf = fs.size();
  std::vector<double*> R0(nf), Sr0(nf), Sc0(nf), junk(nf);
  for (size_t i = 0; i < nf; ++i) {
    R0[i] = fs[i]->R;
    Sr0[i] = fs[i]->Sr;
    Sc0[i] = fs[i]->Sc;
    junk[i] = salloc(h, (int64_t)fs[i]->n * (c0[i] + nc));
  }
  // one pass: F in -> outr, F^T in -> outc
  auto pass = [&](const std::vector<double*>& in, const std::vector<double*>& outr,
                  const std::vector<double*>& outc) {
    for (size_t i = 0; i < nf; ++i) {
      fs[i]->R = in[i];
      fs[i]->Sr = outr[i];
      fs[i]->Sc = outc[i];
    }
    sample(h, fs, c0, nc);
  };
  std::vector<double*> Rr(nf), Rc(nf);
  for (size_t i = 0; i < nf; ++i) {
    Rr[i] = fs[i]->Rr;
    Rc[i] = fs[i]->Rc;
  }
  try {
    for (int it = 0; it < q; ++it) {
      pass(Sr0, junk, Rr);   // R^r = F^T S^r
      pass(Sc0, Rc, junk);   // R^c = F S^c
      pass(Rr, Sr0, junk);   // S^r = F R^r
      pass(Rc, junk, Sc0);   // S^c = F^T R^c
    }
  } catch (...) {
    for (size_t i = 0; i < nf; ++i) {
      fs[i]->R = R0[i];
      fs[i]->Sr = Sr0[i];
      fs[i]->Sc = Sc0[i];
    }
    throw;
  }
  for (size_t i = 0; i < nf; ++i) {
    fs[i]->R = R0[i];
    fs[i]->Sr = Sr0[i];
    fs[i]->Sc = Sc0[i];
  }
}

// unreduced node samples S^r_tau, S^c_tau on all current columns (Alg. 1:
// leaf S - D R, non-leaf stacked reduced children samples minus B R)
void node_samples(Handle& h, const std::vector<NRef>& nodes) {
  std::vector<CopyDesc> cp;
  std::vector<GemmDesc> g;
  for (auto& x : nodes) {
    HFront& F = *x.F;
    HNode& nd = x.n();
    const int d = F.d;
    nd.Sr = salloc(h, (int64_t)nd.mr * d);
    nd.Sc = salloc(h, (int64_t)nd.mc * d);
    if (nd.leaf()) {
      const int m = nd.m();
      cp.push_back(Cp(F.Sr + nd.lo, F.n, nullptr, nd.Sr, m, m, d));
      cp.push_back(Cp(F.Sc + nd.lo, F.n, nullptr, nd.Sc, m, m, d));
      g.push_back(G(nd.D, m, 0, F.rr() + nd.lo, F.n, 0, nd.Sr, m, m, d, m, -1.0, 1.0));
      g.push_back(G(nd.D, m, 1, F.rc() + nd.lo, F.n, 0, nd.Sc, m, m, d, m, -1.0, 1.0));
    } else {
      HNode& a = F.nd[nd.kid[0]];
      HNode& b = F.nd[nd.kid[1]];
      cp.push_back(Cp(a.Srr, a.r, nullptr, nd.Sr, nd.mr, a.r, d));
      cp.push_back(Cp(b.Srr, b.r, nullptr, nd.Sr + a.r, nd.mr, b.r, d));
      cp.push_back(Cp(a.Scr, a.c, nullptr, nd.Sc, nd.mc, a.c, d));
      cp.push_back(Cp(b.Scr, b.c, nullptr, nd.Sc + a.c, nd.mc, b.c, d));
      // S^r: [S_a - B12 R^r_b ; S_b - B21 R^r_a]
      g.push_back(G(nd.B12, a.r, 0, b.Rrr, b.c, 0, nd.Sr, nd.mr, a.r, d, b.c, -1.0, 1.0));
      g.push_back(G(nd.B21, b.r, 0, a.Rrr, a.c, 0, nd.Sr + a.r, nd.mr, b.r, d, a.c, -1.0, 1.0));
      // S^c: [S_a - B21^T R^c_b ; S_b - B12^T R^c_a]
      g.push_back(G(nd.B21, b.r, 1, b.Rcr, b.r, 0, nd.Sc, nd.mc, a.c, d, b.r, -1.0, 1.0));
      g.push_back(G(nd.B12, a.r, 1, a.Rcr, a.r, 0, nd.Sc + a.c, nd.mc, b.c, d, a.r, -1.0, 1.0));
    }
  }
  run_copy(h, cp);
  run_gemm(h, g);
}

// reduced samples and random matrices after the ID: S(J,:), R^r = V^T R,
// R^c = U^T R with U = Pi [I; E] applied as a row gather plus one GEMM
void reduce_nodes(Handle& h, const std::vector<NRef>& nodes) {
  std::vector<CopyDesc> stack, sel;
  std::vector<GemmDesc> g;
  for (auto& x : nodes) {
    HFront& F = *x.F;
    HNode& nd = x.n();
    const int d = F.d;
    nd.Srr = lalloc(h, (int64_t)nd.r * d);
    nd.Scr = lalloc(h, (int64_t)nd.c * d);
    nd.Rrr = lalloc(h, (int64_t)nd.c * d);
    nd.Rcr = lalloc(h, (int64_t)nd.r * d);
    const double *Rin_r, *Rin_c;
    int ld_r, ld_c;
    if (nd.leaf()) {
      Rin_r = F.rr() + nd.lo;
      Rin_c = F.rc() + nd.lo;
      ld_r = ld_c = F.n;
    } else {
      HNode& a = F.nd[nd.kid[0]];
      HNode& b = F.nd[nd.kid[1]];
      double* tr = salloc(h, (int64_t)nd.mc * d);
      double* tc = salloc(h, (int64_t)nd.mr * d);
      stack.push_back(Cp(a.Rrr, a.c, nullptr, tr, nd.mc, a.c, d));
      stack.push_back(Cp(b.Rrr, b.c, nullptr, tr + a.c, nd.mc, b.c, d));
      stack.push_back(Cp(a.Rcr, a.r, nullptr, tc, nd.mr, a.r, d));
      stack.push_back(Cp(b.Rcr, b.r, nullptr, tc + a.r, nd.mr, b.r, d));
      Rin_r = tr; ld_r = nd.mc;
      Rin_c = tc; ld_c = nd.mr;
    }
    sel.push_back(Cp(nd.Sr, nd.mr, nd.dpermr, nd.Srr, nd.r, nd.r, d));
    sel.push_back(Cp(nd.Sc, nd.mc, nd.dpermc, nd.Scr, nd.c, nd.c, d));
    sel.push_back(Cp(Rin_r, ld_r, nd.dpermc, nd.Rrr, nd.c, nd.c, d));
    sel.push_back(Cp(Rin_c, ld_c, nd.dpermr, nd.Rcr, nd.r, nd.r, d));
    if (nd.mc > nd.c)
      g.push_back(G(nd.Ec, nd.mc - nd.c, 1, Rin_r, ld_r, 0, nd.Rrr, nd.c, nd.c, d, nd.mc - nd.c, 1.0, 1.0,
                    nd.dpermc + nd.c));
    if (nd.mr > nd.r)
      g.push_back(G(nd.Er, nd.mr - nd.r, 1, Rin_c, ld_c, 0, nd.Rcr, nd.r, nd.r, d, nd.mr - nd.r, 1.0, 1.0,
                    nd.dpermr + nd.r));
  }
  run_copy(h, stack);
  run_copy(h, sel);
  run_gemm(h, g);
}

// FrontOpDev table for the fronts of one level (element extraction)
FrontOpDev* front_ops(Handle& h, const std::vector<HFront*>& fs) {
  std::vector<FrontOpDev> v;
  for (HFront* F : fs) {
    F->fop = (int)v.size();
    FrontOpDev o{};
    o.A = {F->a_row, F->a_col, F->a_vidx};
    o.val = h.d_val;
    o.n = F->n;
    const FrontPlan& fp = h.P.fr[F->f];
    o.nkids = 0;
    for (size_t k = 0; k < fp.kids.size(); ++k) {
      int c = fp.kids[k];
      if (h.P.fr[c].u == 0) continue;
      o.U[o.nkids] = h.fr[c].U;
      o.hk[o.nkids] = h.fr[c].hidx >= 0 && h.hf[h.fr[c].hidx].lowrank ? h.hf[h.fr[c].hidx].kdev : nullptr;
      o.ldu[o.nkids] = h.fr[c].ldu;
      o.inv[o.nkids] = h.fr[F->f].d_inv[k];
      o.nkids++;
    }
    v.push_back(o);
  }
  return upload(h, v);
}

void compress_level(Handle& h, std::vector<HFront*>& fs, const FrontOpDev* fops, const int* iota) {
  const hssmf_opts& o = h.o;
  // initial samples.  A front starts with as many random columns as its
  // HSS children ended with (at least d0): its random matrix reuses their
  // columns (Eq. (Rmerge), Sec. 4.3), so fewer than that cannot resolve
  // what they already needed.
  h.larena.release();
  h.sarena.release();
  {
    std::vector<int> dinit;
    for (HFront* F : fs) {
      int d = o.d0;
      for (int c : h.P.fr[F->f].kids)
        if (h.P.fr[c].hss) d = std::max(d, h.hf[h.fr[c].hidx].d);
      dinit.push_back(d);
    }
    std::vector<int> c0;
    for (size_t fi = 0; fi < fs.size(); ++fi) {
      HFront* F = fs[fi];
      F->d = 0;
      F->dcap = 0;
      F->R = F->Sr = F->Sc = F->Rr = F->Rc = nullptr;
      grow_samples(h, *F, dinit[fi]);
      F->d = dinit[fi];
      F->rounds = 0;
      F->swaps = 0;
      F->finished = false;
      F->refresh = false;
      // every numeric pass starts from the structure only: buffers of an
      // earlier pass live in memory that the pass has released
      for (auto& nd : F->nd) {
        HNode fresh;
        fresh.lo = nd.lo; fresh.hi = nd.hi; fresh.parent = nd.parent; fresh.height = nd.height;
        fresh.kid[0] = nd.kid[0]; fresh.kid[1] = nd.kid[1];
        nd = std::move(fresh);
      }
      F->Dk = nullptr; F->ipivk = nullptr; F->mk = 0;
      F->Vbark = F->ThT = F->Phi = F->Upd = nullptr;
      F->lowrank = false;
      F->kdev = nullptr;
      F->kR = F->kSr = F->kSc = F->kTh = F->kPhi = nullptr;
      F->kd = 0;
      F->UpdLP = nullptr;
      F->X = F->t1 = F->t2 = nullptr;
      gen_random(h, *F, 0, F->d);
      c0.push_back(0);
    }
    // one sampling pass per distinct starting width
    std::vector<int> widths(dinit);
    std::sort(widths.begin(), widths.end());
    widths.erase(std::unique(widths.begin(), widths.end()), widths.end());
    for (int wd : widths) {
      std::vector<HFront*> grp;
      std::vector<int> gc0;
      for (size_t fi = 0; fi < fs.size(); ++fi)
        if (dinit[fi] == wd) { grp.push_back(fs[fi]); gc0.push_back(0); }
      sample(h, grp, gc0, wd);
      power_iterate(h, grp, gc0, wd);
    }
  }
  int maxh = 0;
  for (HFront* F : fs) maxh = std::max(maxh, F->maxh);
  while (true) {
    for (int hh = 0; hh <= maxh; ++hh) {
      h.sarena.release();
      std::vector<NRef> refresh, cand;
      for (HFront* F : fs) {
        if (F->finished) continue;
        for (int t = 0; t < (int)F->nd.size(); ++t) {
          HNode& nd = F->nd[t];
          if (nd.height != hh || t == F->root) continue;
          if (nd.done) {
            if (F->refresh) refresh.push_back({F, t});
          } else if (nd.leaf() || (F->nd[nd.kid[0]].done && F->nd[nd.kid[1]].done)) {
            cand.push_back({F, t});
          }
        }
      }
      if (refresh.empty() && cand.empty()) continue;
      // element extraction for the candidates (D at leaves, B at parents)
      std::vector<ExtractDesc> ex;
      for (auto& x : cand) {
        HNode& nd = x.n();
        HFront& F = *x.F;
        if (nd.leaf()) {
          nd.mr = nd.mc = nd.m();
          if (!nd.D) {
            nd.D = dalloc(h, (int64_t)nd.m() * nd.m());
            ex.push_back({nd.D, iota + nd.lo, iota + nd.lo, nd.m(), nd.m(), nd.m(), F.fop});
          }
        } else {
          HNode& a = F.nd[nd.kid[0]];
          HNode& b = F.nd[nd.kid[1]];
          nd.mr = a.r + b.r;
          nd.mc = a.c + b.c;
          if (!nd.B12) {  // the children keep their skeletons across growth rounds
            nd.B12 = dalloc(h, (int64_t)a.r * b.c);
            nd.B21 = dalloc(h, (int64_t)b.r * a.c);
            ex.push_back({nd.B12, a.dIr, b.dIc, a.r, b.c, a.r, F.fop});
            ex.push_back({nd.B21, b.dIr, a.dIc, b.r, a.c, b.r, F.fop});
          }
        }
      }
      run_extract(h, ex, fops);
      std::vector<NRef> all = refresh;
      all.insert(all.end(), cand.begin(), cand.end());
      node_samples(h, all);
      // interpolative decompositions of the candidates (both sides): a
      // column-pivoted QR per side, several workgroups per problem, one
      // launch per pivot step (k_id.hip)
      std::vector<int> off(cand.size() + 1, 0);
      for (size_t i = 0; i < cand.size(); ++i) off[i + 1] = off[i] + cand[i].n().mr + cand[i].n().mc;
      int* ibuf = ialloc(h, off.back());
      int* sbuf = sialloc(h, 4 * (int64_t)cand.size());
      std::vector<IDProb> q;
      int maxm = 0, maxd = 0, tmax = 0, wg = 0;
      for (size_t i = 0; i < cand.size(); ++i) {
        HNode& nd = cand[i].n();
        const int d = cand[i].F->d;
        nd.dpermr = ibuf + off[i];
        nd.dpermc = nd.dpermr + nd.mr;
        for (int sd = 0; sd < 2; ++sd) {
          const int m = sd ? nd.mc : nd.mr;
          const int mn = std::min(m, d);
          IDProb pr{};
          pr.S = sd ? nd.Sc : nd.Sr;
          pr.lds = std::max(m, 1);
          pr.W = salloc(h, (int64_t)m * d);
          pr.norms = salloc(h, m);
          pr.alpha = salloc(h, mn);
          pr.P = std::max(1, (m + kIDCols - 1) / kIDCols);
          pr.slots = salloc(h, 4 * (int64_t)pr.P);
          pr.R1 = salloc(h, (int64_t)mn * mn);
          pr.W2 = salloc(h, (int64_t)m * mn);
          pr.perm = sd ? nd.dpermc : nd.dpermr;
          pr.ipos = sialloc(h, m);
          pr.state = sbuf + 4 * i + 2 * sd;
          pr.first = salloc(h, 1);
          pr.active = reinterpret_cast<unsigned char*>(sialloc(h, (m + 3) / 4 + 1));
          pr.m = m;
          pr.d = d;
          pr.wg0 = wg;
          pr.eps = o.rel_tol;
          pr.atol = o.abs_tol;
          wg += pr.P;
          q.push_back(pr);
          maxm = std::max(maxm, m);
          maxd = std::max(maxd, d);
          tmax = std::max(tmax, mn);
        }
      }
      int* derr = nullptr;
      // diagnostics: HSSMF_ID_CENSUS=1 prints one line per ID pass (problem
      // shapes, ranks, pivot-step launches and the pass's wall time)
      static const bool id_census = std::getenv("HSSMF_ID_CENSUS") != nullptr;
      int census_steps = 0;
      double census_t0 = 0.0;
      if (id_census) {
        HIP_CHECK(hipStreamSynchronize(h.st));
        census_t0 = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now().time_since_epoch()).count();
      }
      // The resident kernel's launch plan for the problems qv, ending with
      // the R1 / R2 gathers; false, with nothing launched and qv unchanged,
      // where it does not apply (a problem above 640 samples, or wider than
      // one cooperative launch holds).  Two launch plans:
      //  - all problems on the template of the pass's largest (d, m), in one
      //    cooperative launch, when some problem spans several workgroups
      //    and all workgroups of the pass fit at once;
      //  - else each problem that fits one workgroup of the template its own
      //    (d, m) selects in an ordinary launch of that template (one launch
      //    per template, side by side on st and the auxiliary streams), then
      //    the wider ones on the template of their largest (d, m), in
      //    cooperative launches of at most its capacity, one after another.
      // The results do not depend on the template or the plan.
      auto run_resident = [&](std::vector<IDProb>& qv, int maxd_v, int maxm_v, int*& derr_v) -> bool {
        const int np_all = (int)qv.size();
        if (np_all == 0) return false;
        // forced pivot orders: every problem of the call or none
        const bool forced = qv[0].force != nullptr;
        for (const IDProb& pr : qv)
          REQUIRE((pr.force != nullptr) == forced, HSSMF_EDEVICE, "interpolative decomposition: mixed forced orders");
        const int t_all = id_res_template(maxd_v, maxm_v);
        if (t_all < 0) return false;
        std::vector<int> tpl(np_all, -1), pall(np_all, 1);
        std::vector<int> wide;   // problems wider than one workgroup of their own template
        int cap_all = 0, tot_all = 0, t_wide = -1, cap_wide = 0;
        bool any_all = false;
        const int c_all = id_res_template_candidates(t_all);
        int wd = 0, wm = 0;
        for (int pi = 0; pi < np_all; ++pi) {
          pall[pi] = (qv[pi].m + c_all - 1) / c_all;
          tot_all += std::max(1, pall[pi]);
          any_all |= pall[pi] > 1;
          tpl[pi] = id_res_template(qv[pi].d, qv[pi].m);
          REQUIRE(tpl[pi] >= 0, HSSMF_EDEVICE, "interpolative decomposition: no template for a problem");
          if (qv[pi].m > id_res_template_candidates(tpl[pi])) {
            wide.push_back(pi);
            wd = std::max(wd, qv[pi].d);
            wm = std::max(wm, qv[pi].m);
          }
        }
        if (any_all) cap_all = id_res_template_capacity(t_all);
        if (!(any_all && tot_all <= cap_all) && !wide.empty()) {
          t_wide = id_res_template(wd, wm);
          cap_wide = id_res_template_capacity(t_wide);
          const int c_wide = id_res_template_candidates(t_wide);
          for (int pi : wide)
            if ((qv[pi].m + c_wide - 1) / c_wide > cap_wide) return false;
        }
        const int np = np_all;
        const bool one = any_all && tot_all <= cap_all;
        // workgroups per problem on the template it runs on
        std::vector<bool> is_wide(np, false);
        for (int pi : wide) is_wide[pi] = true;
        if (one) {
          for (int pi = 0; pi < np; ++pi) qv[pi].P = std::max(1, pall[pi]);
        } else {
          const int c_wide = t_wide >= 0 ? id_res_template_candidates(t_wide) : 1;
          for (int pi = 0; pi < np; ++pi)
            qv[pi].P = is_wide[pi] ? std::max(1, (qv[pi].m + c_wide - 1) / c_wide) : 1;
        }
        int wgm = 0;
        std::vector<int> coopp;   // problems with exchange records
        for (int pi = 0; pi < np; ++pi)
          if (qv[pi].P > 1) {
            coopp.push_back(pi);
            wgm += qv[pi].P;
          }
        if (!coopp.empty()) {
          derr_v = sialloc(h, 1);
          double* slots = salloc(h, 6 * (int64_t)wgm);   // per problem 3 x P x (norm, index)
          int o6 = 0;
          for (int pi : coopp) {
            qv[pi].cand = salloc(h, 3 * (int64_t)qv[pi].P * qv[pi].d);
            qv[pi].slots = slots + o6;
            o6 += 6 * qv[pi].P;
          }
          // every exchange record starts empty
          launch_fill(slots, 6 * (int64_t)wgm, std::numeric_limits<double>::quiet_NaN(), h.st);
          HIP_CHECK(hipMemsetAsync(derr_v, 0, sizeof(int), h.st));
        }
        IDProb* dq = upload(h, qv);
        std::vector<int2> wgs;
        if (one) {
          for (int pi = 0; pi < np; ++pi)
            for (int w = 0; w < qv[pi].P; ++w) wgs.push_back(make_int2(pi, w));
          launch_id_res_template(t_all, dq, upload(h, wgs), (int)wgs.size(), true, derr_v, h.st, forced);
        } else {
          // one workgroup each, grouped by template
          std::map<int, std::vector<int2>> single;
          for (int pi = 0; pi < np; ++pi)
            if (!is_wide[pi]) single[tpl[pi]].push_back(make_int2(pi, 0));
          std::vector<std::pair<int, int2*>> launches;   // template, uploaded map
          std::vector<int> counts;
          for (auto& kv : single) {
            launches.emplace_back(kv.first, upload(h, kv.second));
            counts.push_back((int)kv.second.size());
          }
          const int nl = (int)launches.size();
          const int naux = std::max(0, std::min(nl - 1, (int)Handle::kAux));
          if (naux > 0) {
            h.make_aux();
            HIP_CHECK(hipEventRecord(h.ev_fork, h.st));
            for (int a = 0; a < naux; ++a) HIP_CHECK(hipStreamWaitEvent(h.aux[a], h.ev_fork, 0));
          }
          for (int li = 0; li < nl; ++li) {
            hipStream_t ls = li == 0 || naux == 0 ? h.st : h.aux[(li - 1) % naux];
            launch_id_res_template(launches[li].first, dq, launches[li].second, counts[li], false, derr_v, ls, forced);
          }
          for (int a = 0; a < naux; ++a) {
            HIP_CHECK(hipEventRecord(h.ev_join[a], h.aux[a]));
            HIP_CHECK(hipStreamWaitEvent(h.st, h.ev_join[a], 0));
          }
          // the wider problems: a launch lasts as long as its longest
          // problem, so fill them in order of the most pivot steps a
          // problem can take
          std::stable_sort(wide.begin(), wide.end(), [&](int a, int b) {
            return std::min(qv[a].m, qv[a].d) > std::min(qv[b].m, qv[b].d);
          });
          wgs.clear();
          auto flush = [&]() {
            if (wgs.empty()) return;
            launch_id_res_template(t_wide, dq, upload(h, wgs), (int)wgs.size(), true, derr_v, h.st, forced);
            wgs.clear();
          };
          for (int pi : wide) {
            if ((int)wgs.size() + qv[pi].P > cap_wide) flush();
            for (int w = 0; w < qv[pi].P; ++w) wgs.push_back(make_int2(pi, w));
          }
          flush();
        }
        launch_id_finish(dq, np, maxm_v, h.st);
        return true;
      };
      const bool resident = o.id_kernel == HSSMF_ID_RESIDENT && run_resident(q, maxd, maxm, derr);
      const int res_c = resident ? 1 : 0;   // the pass ran on the resident kernel
      if (resident) {
        census_steps = -1;
      } else if (!q.empty()) {
        const int np = (int)q.size();
        int maxp = 0;
        for (auto& pr : q) maxp = std::max(maxp, pr.P);
        const int cap = o.id_kernel == HSSMF_ID_COOPERATIVE ? id_coop_capacity(maxd) : 0;
        if (cap > 0 && wg <= cap) {
          // every problem of the pass resident at once: one cooperative launch
          derr = sialloc(h, 1);
          double* slots = salloc(h, 8 * (int64_t)wg);   // per problem 2 x P x (norm, index, step tag, pad)
          for (int pi = 0; pi < np; ++pi) {
            q[pi].cand = salloc(h, 2 * (int64_t)q[pi].P * q[pi].d);
            q[pi].slots = slots + 8 * (int64_t)q[pi].wg0;
          }
          IDProb* dq = upload(h, q);
          launch_fill(slots, 8 * (int64_t)wg, -1.0, h.st);   // step tags start at -1
          HIP_CHECK(hipMemsetAsync(derr, 0, sizeof(int), h.st));
          std::vector<int2> wgm;
          auto flush = [&]() {
            if (wgm.empty()) return;
            launch_id_coop(dq, upload(h, wgm), (int)wgm.size(), maxd, derr, h.st);
            wgm.clear();
          };
          for (int pi = 0; pi < np; ++pi) {
            if ((int)wgm.size() + q[pi].P > cap) flush();
            for (int w = 0; w < q[pi].P; ++w) wgm.push_back(make_int2(pi, w));
          }
          flush();
          launch_id_finish(dq, np, maxm, h.st);
        } else {
        // done flags that the host reads without a copy back: each problem's
        // stop step sets its flag in mapped host memory
        IdPoll& ip = h.idpoll;
        ip.reserve(np);
        ip.reset();
        volatile int* hd = ip.host;
        for (int pi = 0; pi < np; ++pi) {
          hd[pi] = (q[pi].m == 0 || q[pi].d == 0) ? 1 : 0;   // no pivot step to take
          q[pi].hdone = ip.dev + pi;
        }
        IDProb* dq = upload(h, q);
        // grid of the live problems' workgroups, rebuilt as problems finish
        // so that they stop taking workgroups
        auto wgmap = [&](const std::vector<int>& live, int& nwg) {
          std::vector<int2> wgm;
          for (int pi : live)
            for (int w = 0; w < q[pi].P; ++w) wgm.push_back(make_int2(pi, w));
          nwg = (int)wgm.size();
          return upload(h, wgm);
        };
        std::vector<int> live(np);
        for (int pi = 0; pi < np; ++pi) live[pi] = pi;
        int nwg = 0;
        const int2* dwgm = wgmap(live, nwg);
        launch_id_init(dq, np, wg, maxd, h.st);
        // The stream never drains: every 4 steps the host drops the problems
        // whose flag is set (rebuilding the grid at most every 16 steps) and
        // stops once all are set, while the event ring keeps it at most a
        // few tens of steps ahead of the device.
        int remap = 0;
        for (int t = 0; t <= tmax; ++t) {
          launch_id_step(dq, dwgm, nwg, t, maxd, h.st);
          census_steps = t + 1;
          ip.pace(t, h.st);
          if ((t & 3) == 3 && t < tmax) {
            std::vector<int> nl;
            for (int pi : live)
              if (!hd[pi]) nl.push_back(pi);
            if (nl.empty()) break;
            if (nl.size() < live.size() && t - remap >= 16) {
              live.swap(nl);
              dwgm = wgmap(live, nwg);
              remap = t;
            }
          }
        }
        launch_id_finish(dq, np, maxm, h.st);
        }
      }
      // the pass's results: the wait flag, the stop steps and ranks, the
      // pivot orders, read back through pinned memory with one
      // synchronization
      std::vector<int> sh(4 * cand.size());
      std::vector<int> hbuf(off.back());
      int* pin = h.pinned_ints(1 + sh.size() + hbuf.size());
      pin[0] = 0;
      if (derr) HIP_CHECK(hipMemcpyAsync(pin, derr, sizeof(int), hipMemcpyDeviceToHost, h.st));
      if (!sh.empty())
        HIP_CHECK(hipMemcpyAsync(pin + 1, sbuf, sh.size() * sizeof(int), hipMemcpyDeviceToHost, h.st));
      if (!hbuf.empty())
        HIP_CHECK(hipMemcpyAsync(pin + 1 + sh.size(), ibuf, hbuf.size() * sizeof(int), hipMemcpyDeviceToHost, h.st));
      HIP_CHECK(hipStreamSynchronize(h.st));
      h.stager.sync();
      const int herr = pin[0];
      std::copy(pin + 1, pin + 1 + sh.size(), sh.begin());
      std::copy(pin + 1 + sh.size(), pin + 1 + sh.size() + hbuf.size(), hbuf.begin());
      REQUIRE(herr == 0, HSSMF_EDEVICE, "interpolative decomposition: a workgroup barrier timed out");
      // Strong rank-revealing QR (Gu and Eisenstat, the rank k held fixed)
      // on both IDs of every node that succeeded.  Per round, for each ID
      // still open: one solve R1 [X | Z] = [R2 | I] and the interchange test
      // (largest rho_ij = X_ij^2 + gamma_j^2 |Z_i|^2); an ID whose rho
      // exceeds f^2, with fewer than kSrrqrMaxSwaps interchanges made, moves
      // its selected column i out and its remaining column j in as the last
      // selected one and is factored again in that pivot order (the
      // resident kernel with a forced order), then tested again.  An ID
      // leaves the rounds right after a test, whose solve has left
      // X = R1^{-1} R2 of its final pivot order in W2: the E step below
      // only copies it (x_ready).
      std::vector<char> x_ready(q.size(), 0);
      if (o.srrqr_f > 0.0 && !q.empty()) {
        REQUIRE(resident, HSSMF_EINVAL, "strong RRQR: an ID pass that the resident kernel cannot take");
        const double f2 = o.srrqr_f * o.srrqr_f;
        auto rank_of = [&](int pi) { return sh[4 * (pi / 2) + 1 + 2 * (pi % 2)]; };
        auto host_perm = [&](int pi) {
          const int i = pi / 2;
          return hbuf.data() + off[i] + (pi % 2 ? cand[i].n().mr : 0);
        };
        std::vector<int> live, nsw(q.size(), 0);
        for (size_t i = 0; i < cand.size(); ++i) {
          HFront& F = *cand[i].F;
          HNode& nd = cand[i].n();
          const int r = sh[4 * i + 1], c = sh[4 * i + 3];
          if (!((r <= F.d - o.p || r == nd.mr) && (c <= F.d - o.p || c == nd.mc))) continue;
          for (int sd = 0; sd < 2; ++sd) {
            const int pi = 2 * (int)i + sd;
            if (rank_of(pi) > 0 && rank_of(pi) < q[pi].m) live.push_back(pi);
          }
        }
        IDProb* dq_all = live.empty() ? nullptr : upload(h, q);
        for (int pi : live) x_ready[pi] = 1;
        while (!live.empty()) {
          const int nl = (int)live.size();
          int mk = 0, mm = 0;
          std::vector<TriProb> tp;
          for (int pi : live) {
            const int k = rank_of(pi);
            mk = std::max(mk, k);
            mm = std::max(mm, q[pi].m);
            tp.push_back({q[pi].R1, k, k, q[pi].W2, k, q[pi].m});
          }
          int* didx = upload(h, live);
          launch_srrqr_eye(dq_all, didx, nl, mk, h.st);
          tri_solve_upper_batched(h, tp);
          double* drho = salloc(h, nl);
          int* de = sialloc(h, nl);
          launch_srrqr_test(dq_all, didx, nl, mm, drho, de, h.st);
          int* tpin = h.pinned_ints(3 * nl);
          HIP_CHECK(hipMemcpyAsync(tpin, drho, nl * sizeof(double), hipMemcpyDeviceToHost, h.st));
          HIP_CHECK(hipMemcpyAsync(tpin + 2 * nl, de, nl * sizeof(int), hipMemcpyDeviceToHost, h.st));
          HIP_CHECK(hipStreamSynchronize(h.st));
          h.stager.sync();
          std::vector<double> rho(nl);
          std::vector<int> ev(tpin + 2 * nl, tpin + 3 * nl);
          std::memcpy(rho.data(), tpin, nl * sizeof(double));
          std::vector<int> redo, forder, foff;
          for (int x = 0; x < nl; ++x) {
            const int pi = live[x];
            const int k = rank_of(pi), m = q[pi].m;
            if (!(rho[x] > f2) || nsw[pi] >= kSrrqrMaxSwaps) continue;
            REQUIRE(ev[x] >= 0 && ev[x] < k * (m - k), HSSMF_EDEVICE, "strong RRQR: interchange test out of range");
            const int ii = ev[x] % k, jj = ev[x] / k;
            const int* pp = host_perm(pi);
            foff.push_back((int)forder.size());
            for (int t = 0; t < k; ++t)
              if (t != ii) forder.push_back(pp[t]);
            forder.push_back(pp[k + jj]);
            ++nsw[pi];
            ++cand[pi / 2].F->swaps;
            redo.push_back(pi);
          }
          if (redo.empty()) break;
          int* dorder = upload(h, forder);
          std::vector<IDProb> qs;
          int md = 0, mm2 = 0;
          for (size_t x = 0; x < redo.size(); ++x) {
            IDProb pr = q[redo[x]];
            pr.force = dorder + foff[x];
            pr.kf = rank_of(redo[x]);
            pr.cand = nullptr;
            pr.slots = nullptr;
            md = std::max(md, pr.d);
            mm2 = std::max(mm2, pr.m);
            qs.push_back(pr);
          }
          int* derr2 = nullptr;
          REQUIRE(run_resident(qs, md, mm2, derr2), HSSMF_EINVAL,
                  "strong RRQR: a re-factorization that the resident kernel cannot take");
          // the wait flag, the ranks and the new pivot orders
          size_t tot = 1 + redo.size();
          for (int pi : redo) tot += q[pi].m;
          int* rpin = h.pinned_ints(tot);
          rpin[0] = 0;
          if (derr2) HIP_CHECK(hipMemcpyAsync(rpin, derr2, sizeof(int), hipMemcpyDeviceToHost, h.st));
          size_t at = 1 + redo.size();
          for (size_t x = 0; x < redo.size(); ++x) {
            const IDProb& pr = q[redo[x]];
            HIP_CHECK(hipMemcpyAsync(rpin + 1 + x, pr.state + 1, sizeof(int), hipMemcpyDeviceToHost, h.st));
            HIP_CHECK(hipMemcpyAsync(rpin + at, pr.perm, pr.m * sizeof(int), hipMemcpyDeviceToHost, h.st));
            at += pr.m;
          }
          HIP_CHECK(hipStreamSynchronize(h.st));
          h.stager.sync();
          REQUIRE(rpin[0] == 0, HSSMF_EDEVICE, "strong RRQR: a workgroup barrier timed out");
          at = 1 + redo.size();
          for (size_t x = 0; x < redo.size(); ++x) {
            const int pi = redo[x];
            REQUIRE(rpin[1 + x] == rank_of(pi), HSSMF_EDEVICE, "strong RRQR: a forced re-factorization stopped early");
            std::copy(rpin + at, rpin + at + q[pi].m, host_perm(pi));
            at += q[pi].m;
          }
          live.swap(redo);
        }
      }
      if (id_census && !cand.empty()) {
        const double ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now().time_since_epoch()).count() - census_t0;
        int mlo = 1 << 30, mhi = 0, dlo = 1 << 30, dhi = 0, kmx = 0, fails = 0;
        double work = 0.0;
        for (size_t i = 0; i < cand.size(); ++i) {
          const int d = cand[i].F->d;
          const int ms2[2] = {cand[i].n().mr, cand[i].n().mc};
          for (int sd = 0; sd < 2; ++sd) {
            const int k = sh[4 * i + 1 + 2 * sd], m = ms2[sd];
            mlo = std::min(mlo, m); mhi = std::max(mhi, m);
            dlo = std::min(dlo, d); dhi = std::max(dhi, d);
            kmx = std::max(kmx, k);
            if (!(k <= d - o.p || k == m)) ++fails;
            work += (double)m * d;
          }
        }
        std::fprintf(stderr, "id pass: height %d  problems %zu  m %d..%d  d %d..%d  kmax %d  failed %d  "
                     "steps %d  words %.3g  %.3f ms\n", hh, 2 * cand.size(), mlo, mhi, dlo, dhi, kmx, fails,
                     census_steps, work, ms);
      }
      if (prof::enabled()) {
        // algorithmic flops of the pivot steps: Householder QR of the d x m
        // matrix truncated at k columns, 4dmk - 2k^2(d+m) + 4/3 k^3 per side
        double fl = 0.0;
        for (size_t i = 0; i < cand.size(); ++i) {
          const double d = cand[i].F->d;
          const int ms[2] = {cand[i].n().mr, cand[i].n().mc};
          for (int sd = 0; sd < 2; ++sd) {
            double k = sh[4 * i + 1 + 2 * sd], m = ms[sd];
            fl += 4.0 * d * m * k - 2.0 * k * k * (d + m) + 4.0 / 3.0 * k * k * k;
          }
        }
        prof::add_flops(res_c > 0 ? 4 : 0, fl);   // class 4: the resident kernel
      }
      std::vector<NRef> ok = refresh;
      std::vector<int> ivec;
      std::vector<std::pair<HNode*, int>> ipos;
      for (size_t i = 0; i < cand.size(); ++i) {
        HFront& F = *cand[i].F;
        HNode& nd = cand[i].n();
        const int* b = hbuf.data() + off[i];
        int r = sh[4 * i + 1], c = sh[4 * i + 3];
        bool okr = r <= F.d - o.p || r == nd.mr;
        bool okc = c <= F.d - o.p || c == nd.mc;
        if (!(okr && okc)) continue;
        nd.r = r;
        nd.c = c;
        nd.permr.assign(b, b + nd.mr);
        nd.permc.assign(b + nd.mr, b + nd.mr + nd.mc);
        std::vector<int> base_r, base_c;
        if (nd.leaf()) {
          for (int j = nd.lo; j < nd.hi; ++j) { base_r.push_back(j); base_c.push_back(j); }
        } else {
          HNode& a = F.nd[nd.kid[0]];
          HNode& bb = F.nd[nd.kid[1]];
          base_r = a.Ir; base_r.insert(base_r.end(), bb.Ir.begin(), bb.Ir.end());
          base_c = a.Ic; base_c.insert(base_c.end(), bb.Ic.begin(), bb.Ic.end());
        }
        nd.Er = dalloc(h, (int64_t)(nd.mr - r) * r);
        nd.Ec = dalloc(h, (int64_t)(nd.mc - c) * c);
        nd.Ir.resize(r);
        nd.Ic.resize(c);
        for (int j = 0; j < r; ++j) nd.Ir[j] = base_r[nd.permr[j]];
        for (int j = 0; j < c; ++j) nd.Ic[j] = base_c[nd.permc[j]];
        ipos.push_back({&nd, (int)ivec.size()});
        ivec.insert(ivec.end(), nd.Ir.begin(), nd.Ir.end());
        ivec.insert(ivec.end(), nd.Ic.begin(), nd.Ic.end());
        nd.done = true;
        ok.push_back(cand[i]);
      }
      {
        // E = (R1^{-1} R2)^T for the successful IDs: batched blocked
        // triangular solve (64-row diagonal blocks + GEMM updates), except
        // where the strong RRQR's last test already solved for X
        std::vector<TriProb> tp;
        std::vector<CopyDesc> tc;
        for (size_t i = 0; i < cand.size(); ++i) {
          HNode& nd = cand[i].n();
          if (!nd.done) continue;
          for (int sd = 0; sd < 2; ++sd) {
            const IDProb& pr = q[2 * i + sd];
            const int k = sd ? nd.c : nd.r, nrest = pr.m - k;
            if (k == 0 || nrest == 0) continue;
            if (!x_ready[2 * i + sd]) tp.push_back({pr.R1, k, k, pr.W2, k, nrest});
            tc.push_back(Cp(pr.W2, k, nullptr, sd ? nd.Ec : nd.Er, nrest, nrest, k, 0, 1.0, nullptr, 1));
          }
        }
        tri_solve_upper_batched(h, tp);
        run_copy(h, tc);
      }
      if (!ivec.empty()) {
        int* dI = upload(h, ivec);
        for (auto& pr : ipos) {
          pr.first->dIr = dI + pr.second;
          pr.first->dIc = dI + pr.second + pr.first->r;
        }
      }
      reduce_nodes(h, ok);
    }
    // front roots: extract B between k and q (or the separator root's children)
    std::vector<ExtractDesc> ex;
    for (HFront* F : fs) {
      if (F->finished) continue;
      HNode& rt = F->nd[F->root];
      if (rt.leaf()) {
        if (!rt.D) {
          rt.D = dalloc(h, (int64_t)rt.m() * rt.m());
          ex.push_back({rt.D, iota + rt.lo, iota + rt.lo, rt.m(), rt.m(), rt.m(), F->fop});
        }
        F->finished = true;
        continue;
      }
      HNode& a = F->nd[rt.kid[0]];
      HNode& b = F->nd[rt.kid[1]];
      if (!(a.done && b.done)) continue;
      rt.B12 = dalloc(h, (int64_t)a.r * b.c);
      rt.B21 = dalloc(h, (int64_t)b.r * a.c);
      ex.push_back({rt.B12, a.dIr, b.dIc, a.r, b.c, a.r, F->fop});
      ex.push_back({rt.B21, b.dIr, a.dIc, b.r, a.c, b.r, F->fop});
      F->finished = true;
    }
    run_extract(h, ex, fops);
    bool all = true;
    for (HFront* F : fs) all = all && F->finished;
    if (all) break;
    // adaptive rank: more random vectors for the fronts that are not done
    std::vector<HFront*> grow;
    std::vector<int> c0;
    for (HFront* F : fs) {
      F->refresh = false;
      if (F->finished) continue;
      if (F->d + o.dd > o.d_max) throw Error(HSSMF_ERANK, "HSS compression reached d_max", F->f);
      grow_samples(h, *F, F->d + o.dd);
      gen_random(h, *F, F->d, o.dd);
      c0.push_back(F->d);
      grow.push_back(F);
      F->d += o.dd;
      F->rounds++;
      F->refresh = true;
    }
    sample(h, grow, c0, o.dd);
    power_iterate(h, grow, c0, o.dd);
  }
  if (o.keep_stages) {
    // the random matrix and the samples at the final d, for inspection
    for (HFront* F : fs) {
      const size_t nd = (size_t)F->n * F->d;
      F->kd = F->d;
      F->kR = dalloc(h, (int64_t)nd);
      F->kSr = dalloc(h, (int64_t)nd);
      F->kSc = dalloc(h, (int64_t)nd);
      HIP_CHECK(hipMemcpyAsync(F->kR, F->R, nd * sizeof(double), hipMemcpyDeviceToDevice, h.st));
      HIP_CHECK(hipMemcpyAsync(F->kSr, F->Sr, nd * sizeof(double), hipMemcpyDeviceToDevice, h.st));
      HIP_CHECK(hipMemcpyAsync(F->kSc, F->Sc, nd * sizeof(double), hipMemcpyDeviceToDevice, h.st));
    }
  }
}

// ULV-like factorization of every k-subtree (Sec. 2.3), bottom-up by
// height, then the LU of the merged top block
void ulv_level(Handle& h, std::vector<HFront*>& fs, const int* iota) {
  int maxh = 0;
  for (HFront* F : fs) maxh = std::max(maxh, F->nd[F->k].height);
  auto in_k = [](HFront* F, int t) {
    while (t >= 0 && t != F->k) t = F->nd[t].parent;
    return t == F->k;
  };
  for (int hh = 0; hh <= maxh; ++hh) {
    h.sarena.release();
    std::vector<NRef> L;
    for (HFront* F : fs)
      for (int t = 0; t < (int)F->nd.size(); ++t)
        if (F->nd[t].height == hh && t != F->k && in_k(F, t)) L.push_back({F, t});
    if (L.empty()) continue;
    // dense generators, merged blocks Dbar and Vbar
    std::vector<InterpDesc> ip;
    std::vector<CopyDesc> cp;
    std::vector<GemmDesc> g1, g2;
    for (auto& x : L) {
      HNode& nd = x.n();
      HFront& F = *x.F;
      nd.Ud = dalloc(h, (int64_t)nd.mr * nd.r);
      nd.Vd = dalloc(h, (int64_t)nd.mc * nd.c);
      ip.push_back({nd.Ud, nd.dpermr, nd.Er, nd.mr, nd.r, nd.mr, 0});
      ip.push_back({nd.Vd, nd.dpermc, nd.Ec, nd.mc, nd.c, nd.mc, 0});
      const int m = nd.mr;
      if (nd.leaf()) {
        nd.Dbar = nd.D;
      } else {
        HNode& a = F.nd[nd.kid[0]];
        HNode& b = F.nd[nd.kid[1]];
        nd.Dbar = salloc(h, (int64_t)m * m);
        nd.Vbar = salloc(h, (int64_t)m * nd.c);
        // diagonal blocks: D^ of the children (last r columns of WQ)
        cp.push_back(Cp(a.WQ + (int64_t)a.nl * a.r, a.r, nullptr, nd.Dbar, m, a.r, a.r));
        cp.push_back(Cp(b.WQ + (int64_t)b.nl * b.r, b.r, nullptr, nd.Dbar + a.r + (int64_t)a.r * m, m, b.r, b.r));
        // off-diagonal blocks: B12 V^_b^T and B21 V^_a^T (V^ = last r rows of QV)
        g1.push_back(G(nd.B12, a.r, 0, b.QV + b.nl, b.mr, 1, nd.Dbar + (int64_t)a.r * m, m, a.r, b.r, b.c, 1.0,
                       0.0));
        g1.push_back(G(nd.B21, b.r, 0, a.QV + a.nl, a.mr, 1, nd.Dbar + a.r, m, b.r, a.r, a.c, 1.0, 0.0));
      }
    }
    run_interp(h, ip);
    run_copy(h, cp);
    run_gemm(h, g1);
    for (auto& x : L) {
      HNode& nd = x.n();
      HFront& F = *x.F;
      if (nd.leaf()) {
        nd.Vbar = nd.Vd;
      } else {
        HNode& a = F.nd[nd.kid[0]];
        HNode& b = F.nd[nd.kid[1]];
        // Vbar = diag(V^_a, V^_b) V_tau
        g2.push_back(G(a.QV + a.nl, a.mr, 0, nd.Vd, nd.mc, 0, nd.Vbar, nd.mr, a.r, nd.c, a.c, 1.0, 0.0));
        g2.push_back(G(b.QV + b.nl, b.mr, 0, nd.Vd + a.c, nd.mc, 0, nd.Vbar + a.r, nd.mr, b.r, nd.c, b.c,
                       1.0, 0.0));
      }
    }
    run_gemm(h, g2);
    // W = Omega Dbar: top rows Dbar[perm[r:]] - E Dbar[perm[:r]], bottom Dbar[perm[:r]]
    std::vector<CopyDesc> wc, cc;
    std::vector<GemmDesc> wg;
    std::vector<InterpDesc> eye;
    std::vector<double*> Wt(L.size()), Wb(L.size()), Cb(L.size()), Yb(L.size()), Tb(L.size()), Mb(L.size()),
        M2(L.size());
    std::vector<int> ncomb(L.size());
    int nlmax = 0;
    for (size_t i = 0; i < L.size(); ++i) {
      HNode& nd = L[i].n();
      const int m = nd.mr, r = nd.r, nl = m - r, c = nd.c;
      nd.nl = nl;
      nlmax = std::max(nlmax, nl);
      Wt[i] = salloc(h, (int64_t)std::max(nl, 1) * m);
      Wb[i] = salloc(h, (int64_t)std::max(r, 1) * m);
      wc.push_back(Cp(nd.Dbar, m, nd.dpermr + r, Wt[i], std::max(nl, 1), nl, m));
      wc.push_back(Cp(nd.Dbar, m, nd.dpermr, Wb[i], std::max(r, 1), r, m));
      if (nl > 0 && r > 0)
        wg.push_back(G(nd.Er, nl, 0, nd.Dbar, m, 0, Wt[i], nl, nl, m, r, -1.0, 1.0, nd.dpermr));
      // combined block [W_top^T | W_bot^T | Vbar | I] (m rows): the QR of the
      // first nl columns applies Qtilde^T to the rest
      ncomb[i] = nl + r + c + m;
      Cb[i] = dalloc(h, (int64_t)m * ncomb[i]);
      Yb[i] = salloc(h, (int64_t)m * kPanel);
      Tb[i] = salloc(h, (int64_t)kPanel * kPanel);
      Mb[i] = salloc(h, (int64_t)kPanel * ncomb[i]);
      M2[i] = salloc(h, (int64_t)kPanel * ncomb[i]);
      cc.push_back(Cp(Wt[i], std::max(nl, 1), nullptr, Cb[i], m, m, nl, 0, 1.0, nullptr, 1));
      cc.push_back(Cp(Wb[i], std::max(r, 1), nullptr, Cb[i] + (int64_t)nl * m, m, m, r, 0, 1.0, nullptr, 1));
      cc.push_back(Cp(nd.Vbar, m, nullptr, Cb[i] + (int64_t)(nl + r) * m, m, m, c));
      eye.push_back({Cb[i] + (int64_t)(nl + r + c) * m, iota, nullptr, m, m, m, 0});
    }
    run_copy(h, wc);
    run_gemm(h, wg);
    run_copy(h, cc);
    run_interp(h, eye);
    // blocked Householder QR: 32-column panels, compact-WY trailing updates
    for (int j0 = 0; j0 < nlmax; j0 += kPanel) {
      std::vector<PanelDesc> pd;
      std::vector<GemmDesc> g1, g2, g3;
      for (size_t i = 0; i < L.size(); ++i) {
        HNode& nd = L[i].n();
        const int m = nd.mr;
        if (j0 >= nd.nl) continue;
        const int nb = std::min(kPanel, nd.nl - j0);
        pd.push_back({Cb[i], Yb[i], Tb[i], m, j0, nb, 0});
        const int ntr = ncomb[i] - (j0 + nb);
        if (ntr <= 0) continue;
        double* Ct = Cb[i] + j0 + (int64_t)(j0 + nb) * m;
        g1.push_back(G(Yb[i] + j0, m, 1, Ct, m, 0, Mb[i], kPanel, nb, ntr, m - j0, 1.0, 0.0));
        g2.push_back(G(Tb[i], kPanel, 1, Mb[i], kPanel, 0, M2[i], kPanel, nb, ntr, nb, 1.0, 0.0));
        g3.push_back(G(Yb[i] + j0, m, 0, M2[i], kPanel, 0, Ct, m, m - j0, ntr, nb, -1.0, 1.0));
      }
      int mpx = 0;
      for (auto& q : pd) mpx = std::max(mpx, q.m - q.j0);
      launch_qr_panel(h.stager.put_vec(pd, h.st), (int)pd.size(), mpx, h.st);
      run_gemm(h, g1);
      run_gemm(h, g2);
      run_gemm(h, g3);
    }
    // L = R^T, [D^21 D^] = W_bot Qtilde, [V^1; V^] = Qtilde^T Vbar, Qtilde^T kept
    std::vector<CopyDesc> fin;
    for (size_t i = 0; i < L.size(); ++i) {
      HNode& nd = L[i].n();
      const int m = nd.mr, r = nd.r, nl = nd.nl, c = nd.c;
      nd.L = dalloc(h, (int64_t)std::max(nl, 1) * std::max(nl, 1));
      nd.WQ = dalloc(h, (int64_t)std::max(r, 1) * m);
      fin.push_back(Cp(Cb[i], m, nullptr, nd.L, std::max(nl, 1), nl, nl, 0, 1.0, nullptr, 1));
      fin.push_back(Cp(Cb[i] + (int64_t)nl * m, m, nullptr, nd.WQ, std::max(r, 1), r, m, 0, 1.0, nullptr, 1));
      nd.QV = Cb[i] + (int64_t)(nl + r) * m;
      nd.Q = Cb[i] + (int64_t)(nl + r + c) * m;  // holds Qtilde^T
    }
    run_copy(h, fin);
  }
  // top node k: merged block and its LU
  std::vector<CopyDesc> cp;
  std::vector<GemmDesc> g1, g2;
  std::vector<InterpDesc> ip;
  for (HFront* F : fs) {
    HNode& k = F->nd[F->k];
    const bool has_gen = F->q >= 0;
    if (has_gen) {
      k.Ud = dalloc(h, (int64_t)k.mr * k.r);
      k.Vd = dalloc(h, (int64_t)k.mc * k.c);
      ip.push_back({k.Ud, k.dpermr, k.Er, k.mr, k.r, k.mr, 0});
      ip.push_back({k.Vd, k.dpermc, k.Ec, k.mc, k.c, k.mc, 0});
    }
    if (k.leaf()) {
      F->mk = k.m();
      F->Dk = dalloc(h, (int64_t)F->mk * F->mk);
      cp.push_back(Cp(k.D, F->mk, nullptr, F->Dk, F->mk, F->mk, F->mk));
    } else {
      HNode& a = F->nd[k.kid[0]];
      HNode& b = F->nd[k.kid[1]];
      const int m = a.r + b.r;
      F->mk = m;
      F->Dk = dalloc(h, (int64_t)m * m);
      cp.push_back(Cp(a.WQ + (int64_t)a.nl * a.r, a.r, nullptr, F->Dk, m, a.r, a.r));
      cp.push_back(Cp(b.WQ + (int64_t)b.nl * b.r, b.r, nullptr, F->Dk + a.r + (int64_t)a.r * m, m, b.r, b.r));
      g1.push_back(G(k.B12, a.r, 0, b.QV + b.nl, b.mr, 1, F->Dk + (int64_t)a.r * m, m, a.r, b.r, b.c, 1.0, 0.0));
      g1.push_back(G(k.B21, b.r, 0, a.QV + a.nl, a.mr, 1, F->Dk + a.r, m, b.r, a.r, a.c, 1.0, 0.0));
    }
    F->ipivk = ialloc(h, F->mk);
  }
  run_interp(h, ip);
  run_copy(h, cp);
  run_gemm(h, g1);
  for (HFront* F : fs) {
    HNode& k = F->nd[F->k];
    if (F->q < 0) continue;
    if (k.leaf()) {
      F->Vbark = k.Vd;
    } else {
      HNode& a = F->nd[k.kid[0]];
      HNode& b = F->nd[k.kid[1]];
      F->Vbark = dalloc(h, (int64_t)F->mk * k.c);
      g2.push_back(G(a.QV + a.nl, a.mr, 0, k.Vd, k.mc, 0, F->Vbark, F->mk, a.r, k.c, a.c, 1.0, 0.0));
      g2.push_back(G(b.QV + b.nl, b.mr, 0, k.Vd + a.c, k.mc, 0, F->Vbark + a.r, F->mk, b.r, k.c, b.c, 1.0, 0.0));
    }
  }
  run_gemm(h, g2);
  std::vector<LUFront> lu;
  for (HFront* F : fs) lu.push_back({F->Dk, F->ipivk, F->mk, F->mk, F->mk, F->f});
  blocked_lu(h, lu);
}

// Device table of a front's update matrix in low-rank form (the q-subtree
// in preorder, the leaf of every update row, Theta^T and Phi) for its
// parent's entry extraction (Sec. 4.5)
void build_kid_table(Handle& h, HFront& F) {
  std::vector<int> order, tix(F.nd.size(), -1), stack{F.q};
  while (!stack.empty()) {
    const int t = stack.back();
    stack.pop_back();
    tix[t] = (int)order.size();
    order.push_back(t);
    const HNode& nd = F.nd[t];
    if (!nd.leaf()) {
      stack.push_back(nd.kid[1]);
      stack.push_back(nd.kid[0]);
    }
  }
  std::vector<HssKidNode> tab(order.size());
  std::vector<int> leaf_of(F.u, -1);
  std::vector<CopyDesc> ut_copies;
  for (size_t i = 0; i < order.size(); ++i) {
    const HNode& nd = F.nd[order[i]];
    HssKidNode& k = tab[i];
    k.lo = nd.lo - F.s;
    k.m = nd.m();
    k.r = nd.r;
    k.parent = order[i] == F.q ? -1 : tix[nd.parent];
    k.depth = k.parent < 0 ? 0 : tab[k.parent].depth + 1;   // parents precede children in preorder
    k.kid0 = nd.leaf() ? -1 : tix[nd.kid[0]];
    k.D = nd.leaf() ? nd.D : nullptr;
    k.UT = nullptr;
    if (order[i] != F.q && nd.r > 0) {
      double* ut = dalloc(h, (int64_t)nd.r * nd.m());
      ut_copies.push_back(Cp(nd.Ubig, nd.m(), nullptr, ut, nd.r, nd.r, nd.m(), 0, 1.0, nullptr, 1));
      k.UT = ut;
    }
    k.T12 = nd.T12;
    k.T21 = nd.T21;
    if (nd.leaf())
      for (int r = 0; r < nd.m(); ++r) leaf_of[k.lo + r] = (int)i;
  }
  run_copy(h, ut_copies);
  HssKidDev kd{};
  kd.u = F.u;
  kd.mk = F.mk;
  kd.nnode = (int)tab.size();
  kd.leaf_of = upload(h, leaf_of);
  kd.nodes = upload(h, tab);
  kd.ThT = F.ThT;
  kd.Phi = F.Phi;
  F.kdev = upload(h, std::vector<HssKidDev>{kd});
}

// nested bases U^big, V^big (Eq. nestedUV) of every non-root node, the
// low-rank Schur product and the dense update matrix of each front
void schur_level(Handle& h, std::vector<HFront*>& fs) {
  int maxh = 0;
  std::vector<HFront*> wu;
  for (HFront* F : fs)
    if (F->q >= 0) { wu.push_back(F); maxh = std::max(maxh, F->nd[F->root].height); }
  if (wu.empty()) return;
  // fronts whose update matrix an HSS parent takes in low-rank form
  for (HFront* F : wu) {
    const int par = h.P.fr[F->f].parent;
    F->lowrank = h.o.hss_update == HSSMF_UPDATE_LOWRANK && par >= 0 && h.P.fr[par].hss;
  }
  for (int hh = 0; hh < maxh; ++hh) {
    std::vector<InterpDesc> ip;
    std::vector<GemmDesc> g;
    for (HFront* F : wu)
      for (int t = 0; t < (int)F->nd.size(); ++t) {
        HNode& nd = F->nd[t];
        if (nd.height != hh || t == F->root) continue;
        if (!nd.Ud) {
          nd.Ud = dalloc(h, (int64_t)nd.mr * nd.r);
          nd.Vd = dalloc(h, (int64_t)nd.mc * nd.c);
          ip.push_back({nd.Ud, nd.dpermr, nd.Er, nd.mr, nd.r, nd.mr, 0});
          ip.push_back({nd.Vd, nd.dpermc, nd.Ec, nd.mc, nd.c, nd.mc, 0});
        }
        if (nd.leaf()) {
          nd.Ubig = nd.Ud;
          nd.Vbig = nd.Vd;
        } else {
          HNode& a = F->nd[nd.kid[0]];
          HNode& b = F->nd[nd.kid[1]];
          const int m = nd.m();
          nd.Ubig = dalloc(h, (int64_t)m * nd.r);
          nd.Vbig = dalloc(h, (int64_t)m * nd.c);
          g.push_back(G(a.Ubig, a.m(), 0, nd.Ud, nd.mr, 0, nd.Ubig, m, a.m(), nd.r, a.r, 1.0, 0.0));
          g.push_back(G(b.Ubig, b.m(), 0, nd.Ud + a.r, nd.mr, 0, nd.Ubig + a.m(), m, b.m(), nd.r, b.r, 1.0, 0.0));
          g.push_back(G(a.Vbig, a.m(), 0, nd.Vd, nd.mc, 0, nd.Vbig, m, a.m(), nd.c, a.c, 1.0, 0.0));
          g.push_back(G(b.Vbig, b.m(), 0, nd.Vd + a.c, nd.mc, 0, nd.Vbig + a.m(), m, b.m(), nd.c, b.c, 1.0, 0.0));
        }
      }
    run_interp(h, ip);
    run_gemm(h, g);
  }
  // Theta^T = U_LU^{-T} (Vbar_k B_qk^T) Ubig_q^T ; Phi = L_LU^{-1} P U_k B_kq Vbig_q^T
  h.sarena.release();
  std::vector<GemmDesc> g1, g2, g3;
  std::vector<double*> T1(wu.size()), T3(wu.size());
  for (size_t i = 0; i < wu.size(); ++i) {
    HFront& F = *wu[i];
    HNode& rt = F.nd[F.root];
    HNode& k = F.nd[F.k];
    HNode& q = F.nd[F.q];
    const int mk = F.mk, u = F.u;
    // root children are (k, q): B12 = B_kq (r_k x c_q), B21 = B_qk (r_q x c_k)
    T1[i] = salloc(h, (int64_t)mk * std::max(q.r, 1));  // Vbar_k B_qk^T : mk x r_q
    g1.push_back(G(F.Vbark, mk, 0, rt.B21, q.r, 1, T1[i], mk, mk, q.r, k.c, 1.0, 0.0));
    T3[i] = salloc(h, (int64_t)std::max(k.r, 1) * u);   // B_kq Vbig_q^T : r_k x u
    g1.push_back(G(rt.B12, k.r, 0, q.Vbig, u, 1, T3[i], std::max(k.r, 1), k.r, u, q.c, 1.0, 0.0));
    F.ThT = F.lowrank ? dalloc(h, (int64_t)mk * u) : salloc(h, (int64_t)mk * u);
    F.Phi = F.lowrank ? dalloc(h, (int64_t)mk * u) : salloc(h, (int64_t)mk * u);
    g2.push_back(G(T1[i], mk, 0, q.Ubig, u, 1, F.ThT, mk, mk, u, q.r, 1.0, 0.0));
    g2.push_back(G(k.Ud, mk, 0, T3[i], std::max(k.r, 1), 0, F.Phi, mk, mk, u, k.r, 1.0, 0.0));
  }
  run_gemm(h, g1);
  run_gemm(h, g2);
  for (HFront* F : wu) {
    // Theta^T := U^{-T} Theta^T  (logical lower, non-unit, transposed access)
    tri_solve_many(h, F->Dk, F->mk, F->mk, F->ThT, F->mk, F->u, true, false, true);
    launch_pivots(F->Phi, F->mk, F->u, F->ipivk, F->mk, 0, sialloc(h, F->mk), h.st);
    tri_solve_many(h, F->Dk, F->mk, F->mk, F->Phi, F->mk, F->u, true, true, false);
  }
  if (h.o.keep_stages)
    for (HFront* F : wu) {
      const size_t nb = sizeof(double) * (size_t)F->mk * F->u;
      F->kTh = dalloc(h, (int64_t)F->mk * F->u);
      F->kPhi = dalloc(h, (int64_t)F->mk * F->u);
      HIP_CHECK(hipMemcpyAsync(F->kTh, F->ThT, nb, hipMemcpyDeviceToDevice, h.st));
      HIP_CHECK(hipMemcpyAsync(F->kPhi, F->Phi, nb, hipMemcpyDeviceToDevice, h.st));
    }
  // B12 Vbig_b^T and B21 Vbig_a^T of every non-leaf node of the q-subtrees:
  // the off-diagonal blocks of F22 are Ubig_a times them.  Kept with the
  // factors for a front in low-rank form (entry extraction by its parent),
  // temporaries for the dense expansion otherwise.
  std::vector<GemmDesc> e1;
  for (HFront* F : wu)
    for (int t = 0; t < (int)F->nd.size(); ++t) {
      HNode& nd = F->nd[t];
      if (nd.leaf() || nd.lo < F->s) continue;
      HNode& a = F->nd[nd.kid[0]];
      HNode& b = F->nd[nd.kid[1]];
      const int64_t na = (int64_t)std::max(a.r, 1) * b.m(), nb = (int64_t)std::max(b.r, 1) * a.m();
      nd.T12 = F->lowrank ? dalloc(h, na) : salloc(h, na);
      nd.T21 = F->lowrank ? dalloc(h, nb) : salloc(h, nb);
      e1.push_back(G(nd.B12, a.r, 0, b.Vbig, b.m(), 1, nd.T12, std::max(a.r, 1), a.r, b.m(), b.c, 1.0, 0.0));
      e1.push_back(G(nd.B21, b.r, 0, a.Vbig, a.m(), 1, nd.T21, std::max(b.r, 1), b.r, a.m(), a.c, 1.0, 0.0));
    }
  run_gemm(h, e1, h.gs());
  // dense update matrix (a dense parent, the dense option, or kept for
  // inspection): expand F22 of the q-subtree, subtract Theta^* Phi
  std::vector<HFront*> ex;
  for (HFront* F : wu) {
    F->Upd = nullptr;
    h.fr[F->f].U = nullptr;
    h.fr[F->f].ldu = F->u;
    if (!F->lowrank || h.o.keep_stages) ex.push_back(F);
  }
  for (HFront* F : ex) {
    F->Upd = dalloc(h, (int64_t)F->u * F->u);
    if (!F->lowrank) h.fr[F->f].U = F->Upd;
  }
  std::vector<CopyDesc> cp;
  for (HFront* F : ex)
    for (int t = 0; t < (int)F->nd.size(); ++t) {
      HNode& nd = F->nd[t];
      if (!nd.leaf() || nd.lo < F->s) continue;
      const int o = nd.lo - F->s;
      cp.push_back(Cp(nd.D, nd.m(), nullptr, F->Upd + o + (int64_t)o * F->u, F->u, nd.m(), nd.m()));
    }
  run_copy(h, cp);
  std::vector<GemmDesc> e2;
  for (HFront* F : ex)
    for (int t = 0; t < (int)F->nd.size(); ++t) {
      HNode& nd = F->nd[t];
      if (nd.leaf() || nd.lo < F->s) continue;
      HNode& a = F->nd[nd.kid[0]];
      HNode& b = F->nd[nd.kid[1]];
      // block (a, b) = Ubig_a (B12 Vbig_b^T) ; block (b, a) = Ubig_b (B21 Vbig_a^T)
      const int oa = a.lo - F->s, ob = b.lo - F->s;
      e2.push_back(G(a.Ubig, a.m(), 0, nd.T12, std::max(a.r, 1), 0, F->Upd + oa + (int64_t)ob * F->u, F->u, a.m(),
                     b.m(), a.r, 1.0, 0.0));
      e2.push_back(G(b.Ubig, b.m(), 0, nd.T21, std::max(b.r, 1), 0, F->Upd + ob + (int64_t)oa * F->u, F->u, b.m(),
                     a.m(), b.r, 1.0, 0.0));
    }
  run_gemm(h, e2, h.gs());
  std::vector<GemmDesc> sg;
  for (HFront* F : ex)
    sg.push_back(G(F->ThT, F->mk, 1, F->Phi, F->mk, 0, F->Upd, F->u, F->u, F->u, F->mk, -1.0, 1.0));
  run_gemm(h, sg, h.gs());
  for (HFront* F : wu)
    if (F->lowrank) build_kid_table(h, *F);
}

}  // namespace

// bf16 copy of a (possibly strided) u x u update matrix
static void launch_copy_bf16(Handle& h, const double* U, int ldu, void* dst, int u) {
  double* tmp = h.cur->get<double>((size_t)u * u);
  CopyDesc c{};
  c.src = U; c.dst = tmp; c.m = u; c.n = u; c.lds = ldu; c.ldd = u; c.alpha = 1.0;
  CopyBatch cb{};
  cb.inl[0] = c;
  launch_copy(cb, 1, copy_tiles(c), 0, h.st);
  launch_convert(tmp, dst, (int64_t)u * u, 1, h.st);
}

// per-front norms of Theta, Phi and the update matrix (diagnostics)
static double dev_fro(Handle& h, const double* p, int64_t n) {
  if (!p || n <= 0) return 0.0;
  std::vector<double> v(n);
  HIP_CHECK(hipMemcpyAsync(v.data(), p, n * sizeof(double), hipMemcpyDeviceToHost, h.st));
  HIP_CHECK(hipStreamSynchronize(h.st));
  double s = 0;
  for (double x : v) s += x * x;
  return std::sqrt(s);
}

static void debug_fronts(Handle& h, std::vector<HFront*>& fs) {
  for (HFront* F : fs) {
    int rr = 0;
    for (auto& nd : F->nd) rr = std::max(rr, nd.r);
    std::fprintf(stderr, "front %d s %d u %d rank %d d %d", F->f, F->s, F->u, rr, F->d);
    if (F->q >= 0)
      std::fprintf(stderr, " mk %d |Th| %.6e |Phi| %.6e |U| %.6e |Dk| %.6e", F->mk,
                   dev_fro(h, F->ThT, (int64_t)F->mk * F->u), dev_fro(h, F->Phi, (int64_t)F->mk * F->u),
                   F->Upd ? dev_fro(h, F->Upd, (int64_t)F->u * F->u) : -1.0, dev_fro(h, F->Dk, (int64_t)F->mk * F->mk));
    std::fprintf(stderr, "\n");
  }
}

// -------------------------------------------------------- numeric ---------
void numeric_factor(Handle& h) {
  const Plan& P = h.P;
  // diagnostics: HSSMF_LEVEL_TIMES=1 prints the time of the dense and the
  // HSS part of every elimination-tree level (synchronizing between them)
  static const bool level_times = std::getenv("HSSMF_LEVEL_TIMES") != nullptr;
  auto wall = []() { return std::chrono::duration<double, std::milli>(
                         std::chrono::steady_clock::now().time_since_epoch()).count(); };
  HIP_CHECK(hipMemsetAsync(h.d_info, 0, sizeof(int), h.st));
  for (size_t lev = 0; lev < P.levels.size(); ++lev) {
    const std::vector<int>& ids = P.levels[lev];
    double tl0 = 0.0, tl1 = 0.0;
    if (level_times) {
      HIP_CHECK(hipStreamSynchronize(h.st));
      tl0 = wall();
    }
    // dense fronts
    std::vector<LUFront> lu;
    int64_t total = 0;
    for (int f : ids)
      if (!P.fr[f].hss) total += (int64_t)P.fr[f].n * P.fr[f].n;
    if (total > 0) {
      launch_fill(h.level_buf[lev], total, 0.0, h.st);
      int64_t a0 = -1, a1 = 0;
      for (int f : ids) {
        const FrontRT& R = h.fr[f];
        if (P.fr[f].hss) continue;
        if (a0 < 0) a0 = R.asm_off;
        a1 = R.asm_off + R.asm_cnt;
      }
      if (a0 >= 0) launch_assemble(h.level_buf[lev], h.d_asm_dst + a0, h.d_asm_src + a0, h.d_val, a1 - a0, h.st);
      for (int slot = 0; slot < 2; ++slot) {
        std::vector<EADesc> ea;
        int maxu = 0;
        for (int f : ids) {
          const FrontPlan& fp = P.fr[f];
          if (fp.hss || (int)fp.kids.size() <= slot) continue;
          int c = fp.kids[slot];
          int u = P.fr[c].u;
          if (u == 0) continue;
          ea.push_back({h.fr[c].U, h.fr[f].F, h.fr[f].d_kidmap[slot], u, h.fr[c].ldu, fp.n, 0});
          maxu = std::max(maxu, u);
        }
        if (!ea.empty()) launch_extend_add(h.stager.put_vec(ea, h.st), (int)ea.size(), maxu, h.st);
      }
      for (int f : ids) {
        const FrontPlan& fp = P.fr[f];
        if (fp.hss) continue;
        lu.push_back({h.fr[f].F, h.fr[f].ipiv, fp.s, fp.n, fp.n, f});
      }
      blocked_lu(h, lu);
    }
    if (level_times) {
      HIP_CHECK(hipStreamSynchronize(h.st));
      tl1 = wall();
    }
    // HSS fronts
    std::vector<HFront*> fs;
    for (int f : ids)
      if (P.fr[f].hss) fs.push_back(&h.hf[h.fr[f].hidx]);
    if (!fs.empty()) {
      FrontOpDev* fops = front_ops(h, fs);
      int nmax = 0;
      for (HFront* F : fs) nmax = std::max(nmax, F->n);
      std::vector<int> iota(nmax);
      for (int i = 0; i < nmax; ++i) iota[i] = i;
      int* d_iota = upload(h, iota);
      if (h.o.gemm_prec != HSSMF_PREC_FP64) {
        // low-precision compact copies of the children's update matrices
        const int bf = h.o.gemm_prec == HSSMF_PREC_BF16;
        std::vector<CopyDesc> cv;
        for (HFront* F : fs)
          for (int c : P.fr[F->f].kids) {
            const int u = P.fr[c].u;
            if (u == 0 || !h.fr[c].U) continue;   // a child in low-rank form has no dense copy
            void* lp = h.cur->alloc((size_t)u * u * (bf ? 2 : 4));
            h.fr[c].Ulp = lp;
            if (bf) launch_copy_bf16(h, h.fr[c].U, h.fr[c].ldu, lp, u);
            else cv.push_back(Cp(h.fr[c].U, h.fr[c].ldu, nullptr, lp, u, u, u));
          }
        if (!cv.empty()) {
          int64_t mx = 0;
          for (auto& c : cv) mx = std::max<int64_t>(mx, copy_tiles(c));
          launch_copy(make_batch<CopyDesc, 32>(cv, h.stager, h.st), (int)cv.size(), mx, 1, h.st);
        }
      }
      double tp[4] = {0, 0, 0, 0};
      auto mark = [&](int i) {
        if (!level_times) return;
        HIP_CHECK(hipStreamSynchronize(h.st));
        tp[i] = wall();
      };
      mark(0);
      compress_level(h, fs, fops, d_iota);
      mark(1);
      ulv_level(h, fs, d_iota);
      mark(2);
      schur_level(h, fs);
      mark(3);
      if (level_times && prof::enabled()) {
        double ms[3];
        int64_t nl[3];
        for (int c = 0; c < 3; ++c) prof::read(c, &ms[c], &nl[c], nullptr);
        std::fprintf(stderr, "   kernel classes: ID steps %.2f ms (%lld launches)  GEMM64 %.2f ms (%lld)  GEMMLP %.2f ms\n",
                     ms[0], (long long)nl[0], ms[1], (long long)nl[1], ms[2]);
      }
      if (level_times) {
        int rounds = 0, maxr = 0;
        for (HFront* F : fs) {
          rounds = std::max(rounds, F->rounds);
          for (auto& nd : F->nd) maxr = std::max(maxr, std::max(nd.r, nd.c));
        }
        std::fprintf(stderr, "   hss phases: compress %8.2f ms (rounds %d, max rank %d)  ulv %8.2f ms  schur %8.2f ms\n",
                     tp[1] - tp[0], rounds, maxr, tp[2] - tp[1], tp[3] - tp[2]);
      }
      if (std::getenv("HSSMF_DEBUG")) debug_fronts(h, fs);
    }
    // check for zero pivots after each level
    int info = 0;
    HIP_CHECK(hipMemcpyAsync(&info, h.d_info, sizeof(int), hipMemcpyDeviceToHost, h.st));
    HIP_CHECK(hipStreamSynchronize(h.st));
    h.stager.sync();
    if (info != 0) {
      h.failed_front = info - 1;
      throw Error(HSSMF_ESINGULAR, "zero pivot in front " + std::to_string(info - 1), info - 1);
    }
    if (level_times)
      std::fprintf(stderr, "level %2zu: %5zu fronts (%zu HSS)  dense %8.2f ms  hss %8.2f ms\n", lev, ids.size(),
                   fs.size(), tl1 - tl0, wall() - tl1);
  }
}

}  // namespace hssmf
