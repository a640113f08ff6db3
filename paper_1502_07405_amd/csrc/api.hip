// C ABI (include/hssmf.h): setup of a factorization (plan, uploads, maps,
// HSS trees), numeric refactorization, preconditioner application, the
// outer solvers (iterative refinement, restarted GMRES with modified
// Gram-Schmidt, Sec. 4.6 / Sec. 6.1), transpose solve and adjoint.
#include <algorithm>
#include <chrono>
#include <climits>
#include <cmath>
#include <cstring>
#include <functional>

#include "solver.hpp"
#include "vec.hpp"

using namespace hssmf;

namespace {

double now_ms() {
  return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

template <class T>
T* upload_big(Handle& h, const T* src, size_t n) {
  T* d = h.cur->get<T>(n);
  if (n) HIP_CHECK(hipMemcpy(d, src, n * sizeof(T), hipMemcpyHostToDevice));
  return d;
}
template <class T>
T* upload_big(Handle& h, const std::vector<T>& v) {
  return upload_big(h, v.data(), v.size());
}

int split(std::vector<HNode>& nd, int lo, int hi, int leaf) {
  if (hi - lo <= leaf) {
    HNode x;
    x.lo = lo; x.hi = hi; x.height = 0;
    nd.push_back(x);
    return (int)nd.size() - 1;
  }
  int mid = lo + (hi - lo + 1) / 2;
  int a = split(nd, lo, mid, leaf);
  int b = split(nd, mid, hi, leaf);
  HNode x;
  x.lo = lo; x.hi = hi;
  x.kid[0] = a; x.kid[1] = b;
  x.height = 1 + std::max(nd[a].height, nd[b].height);
  nd.push_back(x);
  int id = (int)nd.size() - 1;
  nd[a].parent = nd[b].parent = id;
  return id;
}

void setup(Handle& h, const hssmf_csr* A) {
  Plan& P = h.P;
  h.cur = &h.arena;
  h.stager.init(size_t(64) << 20);
  const int n = P.n;
  const int64_t nnz = P.nnz;
  h.d_rowptr = upload_big(h, A->rowptr, (size_t)n + 1);
  h.d_colind = upload_big(h, A->colind, (size_t)nnz);
  h.d_val = upload_big(h, A->val, (size_t)nnz);
  // A^T in CSR over the caller's ordering, values through an index
  {
    std::vector<int64_t> tr(n + 1, 0), tv(nnz);
    std::vector<int> tc(nnz), row(nnz);
    for (int i = 0; i < n; ++i)
      for (int64_t e = A->rowptr[i]; e < A->rowptr[i + 1]; ++e) { tr[A->colind[e] + 1]++; row[e] = i; }
    for (int i = 0; i < n; ++i) tr[i + 1] += tr[i];
    std::vector<int64_t> fill(tr.begin(), tr.end() - 1);
    for (int i = 0; i < n; ++i)
      for (int64_t e = A->rowptr[i]; e < A->rowptr[i + 1]; ++e) {
        int64_t p = fill[A->colind[e]]++;
        tc[p] = i;
        tv[p] = e;
      }
    h.d_trowptr = upload_big(h, tr);
    h.d_tcolind = upload_big(h, tc);
    h.d_tvidx = upload_big(h, tv);
    h.d_row = upload_big(h, row);
    h.d_col = h.d_colind;
  }
  h.d_perm = upload_big(h, P.perm);
  h.d_iperm = upload_big(h, P.iperm);
  h.yws = h.arena.get<double>(n);
  h.d_scal = h.arena.get<double>(1024);
  h.gm = gm_dev(h.arena.get<double>(kGmDevDoubles));
  h.gmpoll.init();
  if (!h.werr_h) {
    HIP_CHECK(hipHostMalloc((void**)&h.werr_h, sizeof(int), hipHostMallocMapped | hipHostMallocCoherent));
    HIP_CHECK(hipHostGetDevicePointer((void**)&h.werr_d, h.werr_h, 0));
    *h.werr_h = 0;
  }
  h.d_part = h.arena.get<double>(kDotParts);
  h.d_info = h.arena.get<int>(2);
  h.fr.assign(P.nfront, FrontRT());
  // per-front maps
  for (int f = 0; f < P.nfront; ++f) {
    const FrontPlan& fp = P.fr[f];
    FrontRT& R = h.fr[f];
    R.d_upd = upload_big(h, fp.upd);
    R.w = h.arena.get<double>(std::max(fp.u, 1));
    for (size_t k = 0; k < fp.kids.size(); ++k) {
      R.d_kidmap[k] = upload_big(h, fp.kidmap[k]);
      std::vector<int> inv(fp.n, -1);
      for (size_t t = 0; t < fp.kidmap[k].size(); ++t) inv[fp.kidmap[k][t]] = (int)t;
      R.d_inv[k] = upload_big(h, inv);
    }
  }
  // dense fronts: one buffer per level, assembly maps in level order
  std::vector<int64_t> adst, asrc;
  h.level_buf.assign(P.levels.size(), nullptr);
  for (size_t lev = 0; lev < P.levels.size(); ++lev) {
    int64_t total = 0;
    for (int f : P.levels[lev])
      if (!P.fr[f].hss) total += (int64_t)P.fr[f].n * P.fr[f].n;
    if (total == 0) continue;
    double* buf = h.arena.get<double>(total);
    h.level_buf[lev] = buf;
    int64_t off = 0;
    for (int f : P.levels[lev]) {
      const FrontPlan& fp = P.fr[f];
      if (fp.hss) continue;
      FrontRT& R = h.fr[f];
      R.F = buf + off;
      R.ipiv = h.arena.get<int>(std::max(fp.s, 1));
      R.U = R.F + (int64_t)fp.s * (fp.n + 1);
      R.ldu = fp.n;
      LocalCSR L;
      front_local_csr(P, fp, false, L);
      R.asm_off = (int64_t)adst.size();
      for (int r = 0; r < fp.n; ++r)
        for (int e = L.rowptr[r]; e < L.rowptr[r + 1]; ++e) {
          adst.push_back(off + r + (int64_t)L.col[e] * fp.n);
          asrc.push_back(L.vidx[e]);
        }
      R.asm_cnt = (int64_t)adst.size() - R.asm_off;
      off += (int64_t)fp.n * fp.n;
    }
  }
  h.d_asm_dst = upload_big(h, adst);
  h.d_asm_src = upload_big(h, asrc);
  // HSS fronts
  for (int f = 0; f < P.nfront; ++f) {
    const FrontPlan& fp = P.fr[f];
    if (!fp.hss) continue;
    h.fr[f].hidx = (int)h.hf.size();
    h.hf.emplace_back();
    HFront& F = h.hf.back();
    F.f = f; F.n = fp.n; F.s = fp.s; F.u = fp.u;
    const int leaf = std::max(1, h.o.leaf_size);
    F.k = split(F.nd, 0, fp.s, leaf);
    if (fp.u > 0) {
      F.q = split(F.nd, fp.s, fp.n, leaf);
      HNode rt;
      rt.lo = 0; rt.hi = fp.n;
      rt.kid[0] = F.k; rt.kid[1] = F.q;
      rt.height = 1 + std::max(F.nd[F.k].height, F.nd[F.q].height);
      F.nd.push_back(rt);
      F.root = (int)F.nd.size() - 1;
      F.nd[F.k].parent = F.nd[F.q].parent = F.root;
    } else {
      F.root = F.k;
      F.q = -1;
    }
    F.maxh = F.nd[F.root].height;
    // R is keyed by the row's id in its own system's numbering, so a system
    // factored in a batch draws the same random matrix as on its own
    std::vector<int> orig(fp.n);
    int64_t base = 0;
    if (fp.n > 0 && h.sys_off.size() > 2) {
      const int64_t v = P.perm[fp.lo < fp.hi ? fp.lo : fp.upd[0]];
      base = *(std::upper_bound(h.sys_off.begin(), h.sys_off.end(), v) - 1);
    }
    for (int i = 0; i < fp.s; ++i) orig[i] = (int)(P.perm[fp.lo + i] - base);
    for (int i = 0; i < fp.u; ++i) orig[fp.s + i] = (int)(P.perm[fp.upd[i]] - base);
    F.orig = upload_big(h, orig);
    LocalCSR L, T;
    front_local_csr(P, fp, false, L);
    front_local_csr(P, fp, true, T);
    F.a_row = upload_big(h, L.rowptr);
    F.a_col = upload_big(h, L.col);
    F.a_vidx = upload_big(h, L.vidx);
    F.at_row = upload_big(h, T.rowptr);
    F.at_col = upload_big(h, T.col);
    F.at_vidx = upload_big(h, T.vidx);
  }
  HIP_CHECK(hipDeviceSynchronize());
}

void numeric(Handle& h) {
  HIP_CHECK(hipStreamSynchronize(h.st));
  h.stager.sync();
  // the old factors and the solve operations recorded over them go first,
  // so that nothing refers to released memory if this factorization fails
  h.factor_status = HSSMF_EINVAL;
  for (auto& tr : h.sops)
    for (auto& sw : tr) sw.clear();
  h.drop_graphs();   // the sweeps change with the factors
  h.narena.release();
  h.cur = &h.narena;
  for (Arena* a : {&h.arena, &h.narena, &h.larena, &h.sarena}) a->reset_peak();
  double t0 = now_ms();
  static const bool upload_census = std::getenv("HSSMF_UPLOAD_CENSUS") != nullptr;
  const int64_t p0 = h.stager.n_put, q0 = h.stager.n_put_to;
  try {
    numeric_factor(h);
    const int64_t p1 = h.stager.n_put, q1 = h.stager.n_put_to;
    build_solve_ops(h);
    if (upload_census)
      std::fprintf(stderr, "uploads: numeric factorization %lld ring + %lld direct, solve ops %lld ring + %lld direct\n",
                   (long long)(p1 - p0), (long long)(q1 - q0), (long long)(h.stager.n_put - p1),
                   (long long)(h.stager.n_put_to - q1));
    HIP_CHECK(hipStreamSynchronize(h.st));
  } catch (...) {
    // drain what was enqueued before giving the arenas back; the handle
    // keeps the error, and its solve entry points return it
    (void)hipStreamSynchronize(h.st);
    h.stager.sync();
    for (auto& tr : h.sops)
      for (auto& sw : tr) sw.clear();
    h.larena.release();
    h.sarena.release();
    h.cur = &h.arena;
    try {
      throw;
    } catch (const Error& e) {
      h.factor_status = e.code;
    } catch (const std::bad_alloc&) {
      h.factor_status = HSSMF_ENOMEM;
    } catch (...) {
      h.factor_status = HSSMF_EDEVICE;
    }
    throw;
  }
  h.stager.sync();
  h.larena.release();
  h.sarena.release();
  gemm_census_print();
  h.stats.t_factor_ms = now_ms() - t0;
  h.cur = &h.arena;
  h.factor_status = HSSMF_OK;
  // statistics
  int maxr = 0, maxd = 0, rounds = 0, swaps = 0;
  for (auto& F : h.hf) {
    for (auto& nd : F.nd) maxr = std::max(maxr, std::max(nd.r, nd.c));
    maxd = std::max(maxd, F.d);
    rounds += F.rounds;
    swaps += F.swaps;
  }
  h.stats.srrqr_swaps = swaps;
  h.stats.max_rank = maxr;
  h.stats.max_d = maxd;
  h.stats.growth_rounds = rounds;
  h.stats.factor_bytes = (int64_t)(h.arena.used() + h.narena.used());
  h.stats.peak_bytes = (int64_t)(h.arena.peak() + h.narena.peak() + h.larena.peak() + h.sarena.peak());
  int multi = 0;
  for (auto& a : h.sops)
    for (auto& b : a)
      for (const Op& o : b) multi += o.kind == OP_TRSV && o.ws != nullptr;
  h.stats.trsv_multi_ops = multi;
}

}  // namespace

namespace {
thread_local int g_failed_front = -1;

int guard_impl(Handle* h, const std::function<void()>& fn) {
  try {
    fn();
    return HSSMF_OK;
  } catch (const Error& e) {
    if (e.front >= 0) {
      g_failed_front = e.front;
      if (h) h->failed_front = e.front;
    }
    if (std::getenv("HSSMF_VERBOSE")) std::fprintf(stderr, "hssmf: %s\n", e.what());
    return e.code;
  } catch (const std::bad_alloc&) {
    return HSSMF_ENOMEM;
  } catch (const std::exception& e) {
    if (std::getenv("HSSMF_VERBOSE")) std::fprintf(stderr, "hssmf: %s\n", e.what());
    return HSSMF_EDEVICE;
  }
}

// 2-norms of the systems' parts of a vector (one entry for a single system)
std::vector<double> sys_norms(Handle& h, const double* x) {
  const int ns = (int)h.sys_off.size() - 1;
  if (ns <= 1) return {dnrm2(h, x, h.P.n)};
  std::vector<double> v(ns);
  launch_seg_sumsq(x, h.d_sys_off, ns, h.d_seg, h.st);
  HIP_CHECK(hipMemcpyAsync(v.data(), h.d_seg, sizeof(double) * ns, hipMemcpyDeviceToHost, h.st));
  HIP_CHECK(hipStreamSynchronize(h.st));
  h.stager.sync();
  for (double& e : v) e = std::sqrt(e);
  return v;
}

// largest relative residual over the systems, ||r_s|| / ||b_s||
double max_rel(Handle& h, const double* r, const std::vector<double>& nb) {
  std::vector<double> nr = sys_norms(h, r);
  double rel = 0.0;
  for (size_t s = 0; s < nr.size(); ++s) {
    double q = nb[s] > 0 ? nr[s] / nb[s] : (nr[s] > 0 ? INFINITY : 0.0);
    rel = std::max(rel, q);
  }
  return rel;
}

// Device vectors of one outer solve: carved from a caller-provided block
// (the no-allocation entry point's static scratch) or taken from the
// handle's arena and given back when the solve ends.
struct Ws {
  Handle& h;
  double* base;
  size_t cap, off = 0;
  Arena::Mark mk;
  Ws(Handle& hh, double* b = nullptr, size_t c = 0) : h(hh), base(b), cap(c), mk(hh.arena.mark()) {}
  ~Ws() {
    if (!base) h.arena.reset(mk);
  }
  double* get(size_t n) {
    if (!base) return h.arena.get<double>(n);
    const size_t need = (n + 31) & ~size_t(31);   // 256-byte aligned pieces
    REQUIRE(off + need <= cap, HSSMF_EINVAL, "outer solver: workspace too small");
    double* p = base + off;
    off += need;
    return p;
  }
};

// doubles of workspace the outer solver of the options takes for n unknowns
// (refinement may hand over to GMRES, which then reuses its vectors)
size_t outer_ws_doubles(const hssmf_opts& o, int64_t n) {
  const size_t nn = ((size_t)std::max<int64_t>(n, 1) + 31) & ~size_t(31);
  return nn * (size_t)(std::max(1, std::min(o.restart, kGmMaxRestart)) + 3);
}

// a bounded wait between workgroups of a device kernel that gave up during
// the last solve (read once the stream has been synchronized)
void check_waits(Handle& h) {
  if (h.werr_h && __atomic_load_n(h.werr_h, __ATOMIC_ACQUIRE)) {
    __atomic_store_n(h.werr_h, 0, __ATOMIC_RELEASE);
    throw Error(HSSMF_EDEVICE, "triangular solve: a wait between workgroups gave up");
  }
}

// restarted, left-preconditioned GMRES(m) (Sec. 4.6) with the modified
// Gram-Schmidt Arnoldi process and the Givens rotations on the device; x0 =
// 0 (or the given iterate); stops on the true relative residual
int gmres(Handle& h, int trans, const double* b, double* x, hssmf_info* info, Ws& ws, bool graph,
          bool from_x = false, int its0 = 0) {
  const int n = h.P.n, m = std::max(1, std::min(h.o.restart, kGmMaxRestart));
  double* V = ws.get((size_t)n * (m + 1));
  double* w = ws.get(n);
  double* r = ws.get(n);
  const GmDev& gd = h.gm;
  GmPoll& gp = h.gmpoll;
  const std::vector<double> nbs = sys_norms(h, b);
  const double nb = dnrm2(h, b, n);
  if (!from_x || nb == 0.0) launch_fill(x, n, 0.0, h.st);
  if (nb == 0.0) {
    if (info) { info->iterations = 0; info->rel_residual = 0; }
    return HSSMF_OK;
  }
  int its = 0;
  double rel = 1.0, beta0 = -1.0;
  auto true_res = [&](const double* xx) {
    spmv(h, trans, xx, r, -1.0, 0.0);
    launch_axpy(r, b, n, nullptr, 1.0, 0, h.st);
    return max_rel(h, r, nbs);
  };
  while (its < h.o.max_it) {
    // r = M^{-1} (b - A x)
    spmv(h, trans, x, r, -1.0, 0.0);
    launch_axpy(r, b, n, nullptr, 1.0, 0, h.st);
    apply_inverse(h, trans, r, w, graph);
    double beta = dnrm2(h, w, n);
    if (beta0 < 0) beta0 = beta;
    if (beta == 0.0) break;
    launch_gm_start(V, w, n, beta, gd, m, h.st);  // v0 = w / beta, g = beta e1
    bool done = false;
    // Arnoldi steps with the Gram-Schmidt sweep and the Givens rotations on
    // the device; the host only waits for each step's residual estimate
    // (mapped memory, no stream synchronization) to decide whether to go on
    for (int j = 0; j < m && its < h.o.max_it; ++j) {
      double* vj = V + (size_t)j * n;
      spmv(h, trans, vj, r, 1.0, 0.0);
      apply_inverse(h, trans, r, w, graph);
      const int tag = ++gp.tag;
      if (n <= kArnoldiMaxN) {
        launch_arnoldi(w, V, n, j, gd, gp.dev, tag, h.st);
      } else {
        for (int i = 0; i <= j; ++i) {
          launch_dot(w, V + (size_t)i * n, n, h.d_part, gd.hcol + i, 0, h.st);
          launch_axpy(w, V + (size_t)i * n, n, gd.hcol + i, -1.0, 0, h.st);
        }
        launch_dot(w, w, n, h.d_part, gd.hcol + j + 1, 1, h.st);
        launch_axpy(V + (size_t)(j + 1) * n, w, n, gd.hcol + j + 1, 1.0, 1, h.st);
        launch_givens(j, gd, gp.dev, tag, h.st);
      }
      const double est = gp.wait(tag);
      ++its;
      if (est <= h.o.tol * beta0 || its >= h.o.max_it || j == m - 1) {
        // x_t = x + V y with y from the rotated Hessenberg system
        launch_gm_update(w, x, V, n, j + 1, gd, h.st);
        rel = true_res(w);
        if (rel <= h.o.tol || j == m - 1 || its >= h.o.max_it) {
          HIP_CHECK(hipMemcpyAsync(x, w, sizeof(double) * n, hipMemcpyDeviceToDevice, h.st));
          if (rel <= h.o.tol) done = true;
          break;
        }
      }
    }
    if (done) break;
  }
  HIP_CHECK(hipStreamSynchronize(h.st));
  if (info) { info->iterations = its0 + its; info->rel_residual = rel; }
  return rel <= h.o.tol ? HSSMF_OK : HSSMF_ENOCONV;
}

// Iterative refinement; once the relative residual has failed to fall below
// 0.9 times the previous one on two consecutive steps (the factorization is
// then no contraction, e.g. an HSS preconditioner at a large tolerance), the
// solve hands over to GMRES from the current iterate (Sec. 4.6)
int refine(Handle& h, int trans, const double* b, double* x, hssmf_info* info, Ws& ws, bool graph) {
  const int n = h.P.n;
  const size_t mark = ws.off;
  const Arena::Mark amark = h.arena.mark();
  double* r = ws.get(n);
  double* z = ws.get(n);
  const std::vector<double> nbs = sys_norms(h, b);
  apply_inverse(h, trans, b, x, graph);
  double rel = 0.0, prev = 0.0;
  int it = 0, slow = 0;
  for (;; ++it) {
    spmv(h, trans, x, r, -1.0, 0.0);
    launch_axpy(r, b, n, nullptr, 1.0, 0, h.st);
    rel = max_rel(h, r, nbs);
    slow = (it > 0 && rel > 0.9 * prev) ? slow + 1 : 0;
    prev = rel;
    if (rel <= h.o.tol || slow >= 2 || it >= h.o.max_it) break;
    apply_inverse(h, trans, r, z, graph);
    launch_axpy(x, z, n, nullptr, 1.0, 0, h.st);
  }
  HIP_CHECK(hipStreamSynchronize(h.st));
  if (rel > h.o.tol && slow >= 2) {
    // r and z are dead: GMRES takes their place in the workspace
    ws.off = mark;
    if (!ws.base) h.arena.reset(amark);
    if (info) info->outer_switched = 1;
    return gmres(h, trans, b, x, info, ws, graph, true, it);
  }
  if (info) { info->iterations = it; info->rel_residual = rel; info->failed_front = -1; }
  return rel <= h.o.tol ? HSSMF_OK : HSSMF_ENOCONV;
}

// one right-hand side; ws null: work vectors from the handle's arena
int outer(Handle& h, int trans, const double* b, double* x, hssmf_info* info, double* wsbase = nullptr,
          size_t wscap = 0) {
  if (info) { info->iterations = 0; info->rel_residual = 0; info->failed_front = -1; info->outer_switched = 0; }
  Ws ws(h, wsbase, wscap);
  const bool graph = wsbase == nullptr;   // capturing a graph allocates
  const int rc = h.o.outer == HSSMF_OUTER_GMRES ? gmres(h, trans, b, x, info, ws, graph)
                                                : refine(h, trans, b, x, info, ws, graph);
  check_waits(h);   // both end with the stream synchronized
  return rc;
}

}  // namespace

namespace hssmf {
int outer_solve(Handle& h, int trans, const double* b, double* x, hssmf_info* info, double* ws, size_t wscap) {
  return outer(h, trans, b, x, info, ws, wscap);
}
size_t outer_workspace(const hssmf_opts& o, int64_t n) { return outer_ws_doubles(o, n); }
}  // namespace hssmf

namespace {

// whether p is device memory (else host memory, pinned or pageable)
bool on_device(const void* p) {
  hipPointerAttribute_t a{};
  if (hipPointerGetAttributes(&a, p) != hipSuccess) {
    (void)hipGetLastError();   // pageable host memory is unknown to the runtime
    return false;
  }
  return a.type == hipMemoryTypeDevice || a.type == hipMemoryTypeManaged;
}

// status precedence when several right-hand sides end differently: any hard
// error first, then ENOCONV, then OK
int worse(int a, int b) {
  if (a == HSSMF_OK) return b;
  if (b == HSSMF_OK) return a;
  if (a == HSSMF_ENOCONV) return b;
  return a;
}

// nrhs right-hand sides, host or device, one after another
int outer_many(Handle& h, int trans, int nrhs, const double* b, double* x, hssmf_info* info) {
  const int64_t n = h.P.n;
  const bool bd = on_device(b), xd = on_device(x);
  Arena::Mark mk = h.arena.mark();
  double* bs = bd ? nullptr : h.arena.get<double>((size_t)n);
  double* xs = xd ? nullptr : h.arena.get<double>((size_t)n);
  int st = HSSMF_OK;
  try {
    for (int j = 0; j < nrhs; ++j) {
      const double* bj = b + (size_t)j * n;
      double* xj = x + (size_t)j * n;
      if (!bd) {
        HIP_CHECK(hipMemcpyAsync(bs, bj, sizeof(double) * n, hipMemcpyHostToDevice, h.st));
        bj = bs;
      }
      double* xo = xd ? xj : xs;
      st = worse(st, outer(h, trans, bj, xo, info ? info + j : nullptr));
      if (!xd) {
        HIP_CHECK(hipMemcpyAsync(xj, xs, sizeof(double) * n, hipMemcpyDeviceToHost, h.st));
        HIP_CHECK(hipStreamSynchronize(h.st));
      }
    }
  } catch (...) {
    (void)hipStreamSynchronize(h.st);
    h.arena.reset(mk);
    throw;
  }
  h.arena.reset(mk);
  return st;
}

}  // namespace

extern "C" {

int hssmf_default_opts(hssmf_opts* o) {
  if (!o) return HSSMF_EINVAL;
  std::memset(o, 0, sizeof(*o));
  o->rel_tol = 1e-6;
  o->leaf_size = 64;
  o->min_sep_hss = INT32_MAX;
  o->d0 = 128;
  o->dd = 128;
  o->p = 10;
  o->d_max = 4096;
  o->seed = 0;
  o->gemm_prec = HSSMF_PREC_FP64;
  o->outer = HSSMF_OUTER_IR;
  o->restart = 30;
  o->tol = 1e-10;
  o->max_it = 50;
  o->id_kernel = HSSMF_ID_RESIDENT;
  o->hss_update = HSSMF_UPDATE_DENSE;
  o->power_q = 0;
  o->srrqr_f = 0.0;
  o->use_graph = 0;   // capture after every factorization costs more than replay saves
  return HSSMF_OK;
}

}  // extern "C"

namespace {

bool opts_ok(const hssmf_opts* o) {
  return !(o->leaf_size < 1 || o->d0 < 1 || o->dd < 1 || o->p < 0 || o->d_max < o->d0 || !(o->rel_tol >= 0.0) ||
           o->restart < 1 || o->max_it < 0 || o->gemm_prec < 0 || o->gemm_prec > 2 || o->id_kernel < 0 ||
           o->id_kernel > 2 || o->use_graph < 0 || o->use_graph > 1 ||
           !(o->gemm_tile == 0 || o->gemm_tile == 64 || o->gemm_tile == 65 || o->gemm_tile == 128) ||
           !(o->abs_tol >= 0.0) || o->keep_stages < 0 || o->keep_stages > 1 || o->hss_update < 0 ||
           o->hss_update > 1 || o->power_q < 0 || o->power_q > 4 ||
           (o->power_q > 0 && o->gemm_prec != HSSMF_PREC_FP64) ||
           !(o->srrqr_f == 0.0 || (o->srrqr_f > 1.0 && o->srrqr_f <= 1e300)) ||
           (o->srrqr_f > 0.0 && o->id_kernel != HSSMF_ID_RESIDENT));
}

// a CSR matrix in host memory: the caller's arrays when they are host
// memory, else copies of its device arrays
struct HostCSR {
  hssmf_csr a{};
  std::vector<int64_t> rp;
  std::vector<int32_t> ci;
  std::vector<double> v;
};
// per: values per stored entry (1 real, 2 for a complex (re, im) pair)
int to_host(const hssmf_csr* A, HostCSR& out, int per = 1) {
  out.a = *A;
  out.a.mem = HSSMF_MEM_HOST;
  if (A->mem == HSSMF_MEM_HOST) return HSSMF_OK;
  if (A->mem != HSSMF_MEM_DEVICE || A->n < 0 || !A->rowptr) return HSSMF_EINVAL;
  return guard_impl(nullptr, [&]() {
    out.rp.resize((size_t)A->n + 1);
    HIP_CHECK(hipMemcpy(out.rp.data(), A->rowptr, sizeof(int64_t) * out.rp.size(), hipMemcpyDeviceToHost));
    const int64_t nnz = out.rp[A->n] - out.rp[0];
    REQUIRE(out.rp[0] >= 0 && nnz >= 0, HSSMF_EINVAL, "device CSR: bad rowptr");
    REQUIRE(nnz == 0 || (A->colind && A->val), HSSMF_EINVAL, "device CSR: null arrays");
    out.ci.resize((size_t)out.rp[A->n]);
    out.v.resize((size_t)out.rp[A->n] * per);
    if (!out.ci.empty()) {
      HIP_CHECK(hipMemcpy(out.ci.data(), A->colind, sizeof(int32_t) * out.ci.size(), hipMemcpyDeviceToHost));
      HIP_CHECK(hipMemcpy(out.v.data(), A->val, sizeof(double) * out.v.size(), hipMemcpyDeviceToHost));
    }
    out.a.rowptr = out.rp.data();
    out.a.colind = out.ci.data();
    out.a.val = out.v.data();
  });
}

int factor_impl(const hssmf_csr* A, const hssmf_ordering* ord, const hssmf_opts* opts, void* stream, void** out,
                std::vector<int64_t> sys_off) {
  Handle* h = new (std::nothrow) Handle();
  if (!h) return HSSMF_ENOMEM;
  int rc = guard_impl(h, [&]() {
    double t0 = now_ms();
    // host validation and symbolic analysis first: malformed input is
    // reported without touching the device
    build_plan(A, ord, opts, h->P);
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev == 0) throw Error(HSSMF_EDEVICE, "no HIP device");
    HIP_CHECK(hipGetDevice(&h->device));
    h->o = *opts;
    h->st = static_cast<hipStream_t>(stream);
    h->sys_off = std::move(sys_off);
    setup(*h, A);
    if (h->sys_off.size() > 2) {
      h->d_sys_off = h->arena.get<int64_t>(h->sys_off.size());
      h->d_seg = h->arena.get<double>(h->sys_off.size());
      HIP_CHECK(hipMemcpyAsync(h->d_sys_off, h->sys_off.data(), sizeof(int64_t) * h->sys_off.size(),
                               hipMemcpyHostToDevice, h->st));
      HIP_CHECK(hipStreamSynchronize(h->st));
    }
    h->stats.t_plan_ms = now_ms() - t0;
    h->stats.n = h->P.n;
    h->stats.nfront = h->P.nfront;
    h->stats.n_hss_fronts = (int)h->hf.size();
    numeric(*h);
  });
  if (rc != HSSMF_OK) {
    delete h;
    return rc;
  }
  g_failed_front = -1;
  *out = h;
  return HSSMF_OK;
}

}  // namespace

extern "C" {

int hssmf_factor(const hssmf_csr* A, const hssmf_ordering* ord, const hssmf_opts* opts, void* stream, void** out) {
  if (!out || !A || !ord || !opts) return HSSMF_EINVAL;
  *out = nullptr;
  if (!opts_ok(opts)) return HSSMF_EINVAL;
  HostCSR hc;
  int rc = to_host(A, hc);
  if (rc != HSSMF_OK) return rc;
  return factor_impl(&hc.a, ord, opts, stream, out, {0, (int64_t)std::max(A->n, 0)});
}

int hssmf_factor_batch(int32_t nsys, const hssmf_csr* A, const hssmf_ordering* ord, const hssmf_opts* opts,
                       void* stream, void** out) {
  if (!out || !A || !ord || !opts || nsys < 1) return HSSMF_EINVAL;
  *out = nullptr;
  if (!opts_ok(opts)) return HSSMF_EINVAL;
  // one block-diagonal matrix whose elimination forest has one tree per
  // system, numbered system by system (each system's postorder kept)
  std::vector<HostCSR> hcs(nsys);
  for (int s = 0; s < nsys; ++s) {
    int rc = to_host(A + s, hcs[s]);
    if (rc != HSSMF_OK) return rc;
  }
  std::vector<hssmf_csr> Ah(nsys);
  for (int s = 0; s < nsys; ++s) Ah[s] = hcs[s].a;
  A = Ah.data();
  int64_t n = 0, nnz = 0, nf = 0;
  for (int s = 0; s < nsys; ++s) {
    if (A[s].n < 0 || !A[s].rowptr || (A[s].n > 0 && (!A[s].colind || !A[s].val)) || ord[s].nfront < 0 ||
        !ord[s].sep_ptr || !ord[s].parent || (A[s].n > 0 && !ord[s].perm))
      return HSSMF_EINVAL;
    n += A[s].n;
    nnz += A[s].rowptr[A[s].n];
    nf += ord[s].nfront;
  }
  if (n > INT32_MAX || nf > INT32_MAX) return HSSMF_EINVAL;
  std::vector<int64_t> rowptr(n + 1, 0), off(nsys + 1, 0);
  std::vector<int> col(nnz), perm(n), sep(nf + 1, 0), par(nf);
  std::vector<double> val(nnz);
  int64_t r0 = 0, e0 = 0, f0 = 0;
  for (int s = 0; s < nsys; ++s) {
    const hssmf_csr& a = A[s];
    const hssmf_ordering& o = ord[s];
    const int64_t base = a.rowptr[0];
    for (int i = 0; i < a.n; ++i) rowptr[r0 + i + 1] = e0 + (a.rowptr[i + 1] - base);
    for (int64_t e = 0; e < a.rowptr[a.n] - base; ++e) {
      col[e0 + e] = a.colind[base + e] + (int)r0;
      val[e0 + e] = a.val[base + e];
    }
    for (int i = 0; i < a.n; ++i) perm[r0 + i] = o.perm[i] + (int)r0;
    for (int f = 0; f < o.nfront; ++f) {
      sep[f0 + f + 1] = o.sep_ptr[f + 1] + (int)r0;
      par[f0 + f] = o.parent[f] < 0 ? -1 : o.parent[f] + (int)f0;
    }
    if (o.nfront > 0 && o.sep_ptr[0] != 0) return HSSMF_EINVAL;
    r0 += a.n;
    e0 += a.rowptr[a.n] - base;
    f0 += o.nfront;
    off[s + 1] = r0;
  }
  hssmf_csr ca{(int32_t)n, rowptr.data(), col.data(), val.data(), HSSMF_MEM_HOST};
  hssmf_ordering co{perm.data(), (int32_t)nf, sep.data(), par.data()};
  return factor_impl(&ca, &co, opts, stream, out, off);
}

int hssmf_factor_z(const hssmf_csr* A, const hssmf_ordering* ord, const hssmf_opts* opts, void* stream,
                   void** out) {
  if (!out || !A || !ord || !opts) return HSSMF_EINVAL;
  *out = nullptr;
  if (!opts_ok(opts)) return HSSMF_EINVAL;
  HostCSR hc;
  int rc = to_host(A, hc, 2);
  if (rc != HSSMF_OK) return rc;
  const hssmf_csr& a = hc.a;
  if (a.n < 0 || a.n > INT32_MAX / 2 || !a.rowptr || ord->nfront < 0 || !ord->sep_ptr || !ord->parent ||
      (a.n > 0 && (!a.colind || !a.val || !ord->perm)))
    return HSSMF_EINVAL;
  const int64_t base = a.rowptr[0];
  const int64_t nnz = a.rowptr[a.n] - base;
  if (base < 0 || nnz < 0) return HSSMF_EINVAL;
  for (int i = 0; i < a.n; ++i)
    if (a.rowptr[i + 1] < a.rowptr[i]) return HSSMF_EINVAL;
  // the real-equivalent form: unknown j becomes 2j (real part) and 2j + 1
  // (imaginary part); entry alpha + i beta becomes [alpha -beta; beta alpha]
  const int n2 = 2 * a.n;
  std::vector<int64_t> rp(n2 + 1, 0), zrow(a.n + 1);
  std::vector<int32_t> ci(4 * nnz);
  std::vector<double> v(4 * nnz);
  for (int i = 0; i < a.n; ++i) {
    const int64_t e0 = a.rowptr[i] - base, len = a.rowptr[i + 1] - a.rowptr[i];
    zrow[i] = e0;
    rp[2 * i + 1] = rp[2 * i] + 2 * len;
    rp[2 * i + 2] = rp[2 * i + 1] + 2 * len;
    for (int64_t t = 0; t < len; ++t) {
      const int j = a.colind[base + e0 + t];
      if (j < 0 || j >= a.n) return HSSMF_EINVAL;
      const double re = a.val[2 * (base + e0 + t)], im = a.val[2 * (base + e0 + t) + 1];
      const int64_t r0 = rp[2 * i] + 2 * t, r1 = rp[2 * i + 1] + 2 * t;
      ci[r0] = 2 * j;
      ci[r0 + 1] = 2 * j + 1;
      v[r0] = re;
      v[r0 + 1] = -im;
      ci[r1] = 2 * j;
      ci[r1 + 1] = 2 * j + 1;
      v[r1] = im;
      v[r1 + 1] = re;
    }
  }
  zrow[a.n] = nnz;
  std::vector<int32_t> perm(n2), sep(ord->nfront + 1), par(ord->parent, ord->parent + ord->nfront);
  for (int k = 0; k < a.n; ++k) {
    const int p = ord->perm[k];
    if (p < 0 || p >= a.n) return HSSMF_EINVAL;
    perm[2 * k] = 2 * p;
    perm[2 * k + 1] = 2 * p + 1;
  }
  for (int f = 0; f <= ord->nfront; ++f) {
    if (ord->sep_ptr[f] < 0 || ord->sep_ptr[f] > a.n) return HSSMF_EINVAL;
    sep[f] = 2 * ord->sep_ptr[f];
  }
  hssmf_csr ca{n2, rp.data(), ci.data(), v.data(), HSSMF_MEM_HOST};
  hssmf_ordering co{perm.data(), ord->nfront, sep.data(), par.data()};
  rc = factor_impl(&ca, &co, opts, stream, out, {0, (int64_t)n2});
  if (rc == HSSMF_OK) {
    Handle* h = static_cast<Handle*>(*out);
    h->zexp = true;
    h->zrow = std::move(zrow);
    rc = guard_impl(h, [&]() {
      h->d_zrow = h->arena.get<int64_t>(h->zrow.size());
      HIP_CHECK(hipMemcpyAsync(h->d_zrow, h->zrow.data(), sizeof(int64_t) * h->zrow.size(), hipMemcpyHostToDevice,
                               h->st));
      HIP_CHECK(hipStreamSynchronize(h->st));
    });
    if (rc != HSSMF_OK) {
      hssmf_destroy(h);
      *out = nullptr;
    }
  }
  return rc;
}

int hssmf_refactor_z_device(void* hv, const double* val_dev) {
  Handle* h = static_cast<Handle*>(hv);
  if (!h || !val_dev || !h->zexp || !h->d_zrow) return HSSMF_EINVAL;
  return guard_impl(h, [&]() {
    launch_zexpand(h->d_val, val_dev, h->d_zrow, (int)h->zrow.size() - 1, h->st);
    numeric(*h);
  });
}

int hssmf_refactor_z(void* hv, const double* val) {
  Handle* h = static_cast<Handle*>(hv);
  if (!h || !val || !h->zexp) return HSSMF_EINVAL;
  return guard_impl(h, [&]() {
    const int n = (int)h->zrow.size() - 1;
    std::vector<double> v((size_t)h->P.nnz);
    int64_t r = 0;
    for (int i = 0; i < n; ++i) {
      const int64_t e0 = h->zrow[i], len = h->zrow[i + 1] - e0;
      for (int64_t t = 0; t < len; ++t) {   // the real part's row
        v[r + 2 * t] = val[2 * (e0 + t)];
        v[r + 2 * t + 1] = -val[2 * (e0 + t) + 1];
      }
      r += 2 * len;
      for (int64_t t = 0; t < len; ++t) {   // the imaginary part's row
        v[r + 2 * t] = val[2 * (e0 + t) + 1];
        v[r + 2 * t + 1] = val[2 * (e0 + t)];
      }
      r += 2 * len;
    }
    REQUIRE(r == h->P.nnz, HSSMF_EDEVICE, "complex refactorization: pattern size mismatch");
    HIP_CHECK(hipMemcpyAsync(h->d_val, v.data(), sizeof(double) * v.size(), hipMemcpyHostToDevice, h->st));
    HIP_CHECK(hipStreamSynchronize(h->st));
    numeric(*h);
  });
}

int hssmf_systems(void* hv, int64_t* off, int32_t cap) {
  Handle* h = static_cast<Handle*>(hv);
  if (!h || (cap > 0 && !off)) return HSSMF_EINVAL;
  const int ns = (int)h->sys_off.size() - 1;
  for (int i = 0; i <= ns && i < cap; ++i) off[i] = h->sys_off[i];
  return ns;
}

int hssmf_refactor(void* hv, const double* val) {
  Handle* h = static_cast<Handle*>(hv);
  if (!h || !val) return HSSMF_EINVAL;
  return guard_impl(h, [&]() {
    HIP_CHECK(hipMemcpyAsync(h->d_val, val, sizeof(double) * h->P.nnz, hipMemcpyHostToDevice, h->st));
    numeric(*h);
  });
}

int hssmf_refactor_device(void* hv, const double* val_dev) {
  Handle* h = static_cast<Handle*>(hv);
  if (!h || !val_dev) return HSSMF_EINVAL;
  return guard_impl(h, [&]() {
    HIP_CHECK(hipMemcpyAsync(h->d_val, val_dev, sizeof(double) * h->P.nnz, hipMemcpyDeviceToDevice, h->st));
    numeric(*h);
  });
}

int hssmf_apply(void* hv, int32_t trans, const double* x, double* y) {
  Handle* h = static_cast<Handle*>(hv);
  if (!h || !x || !y || (trans != 0 && trans != 1)) return HSSMF_EINVAL;
  if (h->factor_status != HSSMF_OK) return h->factor_status;
  return guard_impl(h, [&]() {
    apply_inverse(*h, trans, x, y);
    HIP_CHECK(hipStreamSynchronize(h->st));
    h->stager.sync();
    check_waits(*h);
  });
}

int hssmf_solve(void* hv, int32_t nrhs, const double* b, double* x, hssmf_info* info) {
  Handle* h = static_cast<Handle*>(hv);
  if (!h || nrhs < 0 || (nrhs > 0 && (!b || !x))) return HSSMF_EINVAL;
  if (h->factor_status != HSSMF_OK) return h->factor_status;
  int out = HSSMF_OK;
  int rc = guard_impl(h, [&]() { out = outer_many(*h, 0, nrhs, b, x, info); });
  return rc != HSSMF_OK ? rc : out;
}

int hssmf_solve_transpose(void* hv, int32_t nrhs, const double* g, double* lam, hssmf_info* info) {
  Handle* h = static_cast<Handle*>(hv);
  if (!h || nrhs < 0 || (nrhs > 0 && (!g || !lam))) return HSSMF_EINVAL;
  if (h->factor_status != HSSMF_OK) return h->factor_status;
  int out = HSSMF_OK;
  int rc = guard_impl(h, [&]() { out = outer_many(*h, 1, nrhs, g, lam, info); });
  return rc != HSSMF_OK ? rc : out;
}

int hssmf_solve_batch(void* hv, const double* const* b, double* const* x, hssmf_info* info) {
  Handle* h = static_cast<Handle*>(hv);
  if (!h || !b || !x) return HSSMF_EINVAL;
  const int ns = (int)h->sys_off.size() - 1;
  for (int s = 0; s < ns; ++s)
    if (h->sys_off[s + 1] > h->sys_off[s] && (!b[s] || !x[s])) return HSSMF_EINVAL;
  if (h->factor_status != HSSMF_OK) return h->factor_status;
  int out = HSSMF_OK;
  int rc = guard_impl(h, [&]() {
    // pack the systems' right-hand sides back to back, solve once, unpack
    const int64_t n = h->P.n;
    Arena::Mark mk = h->arena.mark();
    double* bb = h->arena.get<double>((size_t)n);
    double* xx = h->arena.get<double>((size_t)n);
    auto seg = [&](int s) { return (size_t)(h->sys_off[s + 1] - h->sys_off[s]); };
    try {
      for (int s = 0; s < ns; ++s)
        if (seg(s))
          HIP_CHECK(hipMemcpyAsync(bb + h->sys_off[s], b[s], sizeof(double) * seg(s),
                                   on_device(b[s]) ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, h->st));
      out = outer(*h, 0, bb, xx, info);
      for (int s = 0; s < ns; ++s)
        if (seg(s))
          HIP_CHECK(hipMemcpyAsync(x[s], xx + h->sys_off[s], sizeof(double) * seg(s),
                                   on_device(x[s]) ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, h->st));
      HIP_CHECK(hipStreamSynchronize(h->st));
    } catch (...) {
      (void)hipStreamSynchronize(h->st);
      h->arena.reset(mk);
      throw;
    }
    h->arena.reset(mk);
  });
  return rc != HSSMF_OK ? rc : out;
}

int hssmf_adjoint(void* hv, const double* x, const double* g, double* dl_db, double* dl_dval, hssmf_info* info) {
  Handle* h = static_cast<Handle*>(hv);
  if (!h || !x || !g || !dl_db || !dl_dval) return HSSMF_EINVAL;
  if (h->factor_status != HSSMF_OK) return h->factor_status;
  int out = HSSMF_OK;
  int rc = guard_impl(h, [&]() {
    out = outer(*h, 1, g, dl_db, info);
    launch_adjoint_grad(h->d_row, h->d_col, dl_db, x, dl_dval, h->P.nnz, h->st);
    HIP_CHECK(hipStreamSynchronize(h->st));
  });
  return rc != HSSMF_OK ? rc : out;
}

int hssmf_stats_get(void* hv, hssmf_stats* s) {
  Handle* h = static_cast<Handle*>(hv);
  if (!h || !s) return HSSMF_EINVAL;
  *s = h->stats;
  return HSSMF_OK;
}

int hssmf_hss_ranks(void* hv, int32_t* out, int32_t cap) {
  Handle* h = static_cast<Handle*>(hv);
  if (!h || (cap > 0 && !out)) return HSSMF_EINVAL;
  int i = 0;
  for (auto& F : h->hf) {
    if (i < cap) {
      int mr = 0, mc = 0;
      for (auto& nd : F.nd) { mr = std::max(mr, nd.r); mc = std::max(mc, nd.c); }
      int32_t* o = out + 5 * i;
      o[0] = F.f; o[1] = mr; o[2] = mc; o[3] = F.d; o[4] = F.rounds;
    }
    ++i;
  }
  return i;
}

int hssmf_front_data(void* hv, int32_t front, int32_t what, double* out, int64_t cap, int32_t* dims) {
  Handle* h = static_cast<Handle*>(hv);
  if (!h || !dims || (cap > 0 && !out)) return HSSMF_EINVAL;
  if (h->factor_status != HSSMF_OK) return h->factor_status;
  if (front < 0 || front >= h->P.nfront || h->fr[front].hidx < 0) return HSSMF_EINVAL;
  const HFront& F = h->hf[h->fr[front].hidx];
  const double* src = nullptr;
  int rows = 0, cols = 0;
  switch (what) {
    case HSSMF_STAGE_RANDOM: src = F.kR; rows = F.n; cols = F.kd; break;
    case HSSMF_STAGE_SAMPLES_ROW: src = F.kSr; rows = F.n; cols = F.kd; break;
    case HSSMF_STAGE_SAMPLES_COL: src = F.kSc; rows = F.n; cols = F.kd; break;
    case HSSMF_STAGE_THETA_T: src = F.kTh; rows = F.mk; cols = F.u; break;
    case HSSMF_STAGE_PHI: src = F.kPhi; rows = F.mk; cols = F.u; break;
    case HSSMF_STAGE_UPDATE: src = F.Upd; rows = F.u; cols = F.u; break;
    default: return HSSMF_EINVAL;
  }
  if (!src && (int64_t)rows * cols > 0) return HSSMF_EINVAL;   // not kept (keep_stages off)
  dims[0] = rows;
  dims[1] = cols;
  const int64_t nel = (int64_t)rows * cols;
  if (cap < nel || nel == 0) return HSSMF_OK;
  return guard_impl(h, [&]() {
    HIP_CHECK(hipStreamSynchronize(h->st));
    HIP_CHECK(hipMemcpy(out, src, sizeof(double) * (size_t)nel, hipMemcpyDeviceToHost));
  });
}

int hssmf_measure_peaks(void* stream, hssmf_peaks* out) {
  if (!out) return HSSMF_EINVAL;
  return guard_impl(nullptr, [&]() {
    measure_peaks(static_cast<hipStream_t>(stream), &out->hbm_GBps, &out->fp64_valu_TFLOPs, &out->fp64_mfma_TFLOPs);
  });
}

int hssmf_last_failed_front(void* hv) {
  Handle* h = static_cast<Handle*>(hv);
  return h ? h->failed_front : g_failed_front;
}

void hssmf_destroy(void* hv) {
  Handle* h = static_cast<Handle*>(hv);
  if (!h) return;
  (void)hipStreamSynchronize(h->st);
  delete h;
  arena_trim_cache();
}

const char* hssmf_strerror(int code) {
  switch (code) {
    case HSSMF_OK: return "ok";
    case HSSMF_EINVAL: return "invalid argument";
    case HSSMF_ENOMEM: return "out of memory";
    case HSSMF_ESINGULAR: return "zero pivot";
    case HSSMF_ERANK: return "HSS rank exceeds d_max";
    case HSSMF_ENOCONV: return "no convergence";
    case HSSMF_EDEVICE: return "device error";
    case HSSMF_ETOOBIG: return "problem too large for the no-allocation scratch";
  }
  return "unknown status";
}

}  // extern "C"
