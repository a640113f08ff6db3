// Forward / backward sweeps of the multifrontal solve (Sec. 3.3) with ULV
// solves of the HSS fronts (Sec. 2.3), and their transposes.
//
// Every buffer the sweeps touch has a fixed address once the factorization
// is done, so the launches (with their descriptor arrays) are recorded once
// per factorization and replayed for every application of M^{-1}.
#include <algorithm>
#include <cstring>

#include "solver.hpp"
#include "vec.hpp"

namespace hssmf {

namespace {

// descriptor arrays of all recorded launches go into one host blob that is
// uploaded once; ops hold offsets until the blob has a device address
struct Blob {
  std::vector<char> bytes;
  template <class T>
  const void* add(const std::vector<T>& v) {
    size_t off = (bytes.size() + 255) / 256 * 256;
    bytes.resize(off + v.size() * sizeof(T));
    std::memcpy(bytes.data() + off, v.data(), v.size() * sizeof(T));
    return reinterpret_cast<const void*>(off);
  }
};

struct Rec {
  Handle& h;
  std::vector<Op>& ops;
  Blob& blob;
  template <class T>
  const void* upload(Handle&, const std::vector<T>& v) { return blob.add(v); }
  void gemv(const std::vector<GemvDesc>& v) {
    std::vector<GemvDesc> w;
    int64_t mx = 0;
    for (auto& g : v)
      if (g.rows > 0 && g.cols > 0) {
        w.push_back(g);
        mx = std::max<int64_t>(mx, g.trans ? (g.cols + 3) / 4 : (g.rows + 15) / 16);
      } else if (g.overwrite && (g.trans ? g.cols : g.rows) > 0) {
        // an empty product still has to clear its output
        GemvDesc z = g;
        z.alpha = 0.0;
        z.cols = std::max(z.cols, 1);
        z.rows = std::max(z.rows, 1);
        w.push_back(z);
        mx = std::max<int64_t>(mx, z.trans ? (z.cols + 3) / 4 : (z.rows + 15) / 16);
      }
    if (!w.empty()) ops.push_back({OP_GEMV, upload(h, w), (int)w.size(), mx});
  }
  void copy(const std::vector<CopyDesc>& v) {
    std::vector<CopyDesc> w;
    int64_t mx = 0;
    for (auto& c : v)
      if (c.m > 0 && c.n > 0) { w.push_back(c); mx = std::max<int64_t>(mx, copy_tiles(c)); }
    if (!w.empty()) ops.push_back({OP_COPY, upload(h, w), (int)w.size(), mx});
  }
  void trsv(const std::vector<TrsvDesc>& v, int kind) {
    std::vector<TrsvDesc> w;
    int64_t ms = 0;
    for (auto& t : v)
      if (t.s > 0) { w.push_back(t); ms = std::max<int64_t>(ms, t.s); }
    if (w.empty()) return;
    Op o{OP_TRSV, upload(h, w), (int)w.size(), kind + 16 * ms};
    // long systems: one workgroup per block of 64 entries; their launch,
    // ticket and flag words travel zeroed in the blob (an offset until the
    // blob is on the device, never 0: the descriptors precede them)
    if (trsv_multi_use((int)w.size(), kind, (int)ms)) {
      const size_t nws = 3 + w.size() * (size_t)((ms + 63) / 64 + 1);
      o.ws = reinterpret_cast<int*>(const_cast<void*>(upload(h, std::vector<int>(nws, 0))));
    }
    ops.push_back(o);
  }
  void rhs(const std::vector<RhsDesc>& v, int mx) {
    if (!v.empty()) ops.push_back({OP_RHS, upload(h, v), (int)v.size(), mx});
  }
};

GemvDesc GV(const double* M, int ld, int rows, int cols, int trans, const double* x, double* y, double alpha,
            int overwrite = 0, const int* xmap = nullptr, const int* ymap = nullptr) {
  GemvDesc g{};
  g.M = M; g.ld = ld; g.rows = rows; g.cols = cols; g.trans = trans;
  g.x = x; g.y = y; g.alpha = alpha; g.overwrite = overwrite; g.xmap = xmap; g.ymap = ymap;
  return g;
}

CopyDesc CV(const double* src, const int* rmap, double* dst, int m, int acc = 0, double alpha = 1.0) {
  CopyDesc c{};
  c.src = src; c.dst = dst; c.rmap = rmap; c.m = m; c.n = 1; c.lds = std::max(m, 1); c.ldd = std::max(m, 1);
  c.accumulate = acc; c.alpha = alpha;
  return c;
}

struct NR {
  HFront* F;
  int t;
  double* xv;  // the front's in-place vector (s entries)
};

bool in_k(HFront* F, int t) {
  while (t >= 0 && t != F->k) t = F->nd[t].parent;
  return t == F->k;
}

// ULV solve of F11 z = b in place on xv (per front), all fronts together
void ulv_solve_rec(Rec& R, std::vector<std::pair<HFront*, double*>>& fs) {
  int maxh = 0;
  for (auto& p : fs) maxh = std::max(maxh, p.first->nd[p.first->k].height);
  auto nodes_at = [&](int hh) {
    std::vector<NR> v;
    for (auto& p : fs)
      for (int t = 0; t < (int)p.first->nd.size(); ++t)
        if (p.first->nd[t].height == hh && t != p.first->k && in_k(p.first, t)) v.push_back({p.first, t, p.second});
    return v;
  };
  auto bbar_of = [](NR& x) -> double* {
    HNode& nd = x.F->nd[x.t];
    return nd.leaf() ? x.xv + nd.lo : nd.bbar;
  };
  // merged right-hand side of a non-leaf: [chat_a - B12 w_b; chat_b - B21 w_a]
  auto merge = [&](std::vector<NR>& v) {
    std::vector<CopyDesc> c;
    std::vector<GemvDesc> g;
    for (auto& x : v) {
      HNode& nd = x.F->nd[x.t];
      if (nd.leaf()) continue;
      HNode& a = x.F->nd[nd.kid[0]];
      HNode& b = x.F->nd[nd.kid[1]];
      c.push_back(CV(a.cbot, nullptr, nd.bbar, a.r));
      c.push_back(CV(b.cbot, nullptr, nd.bbar + a.r, b.r));
      g.push_back(GV(nd.B12, std::max(a.r, 1), a.r, b.c, 0, b.w, nd.bbar, -1.0));
      g.push_back(GV(nd.B21, std::max(b.r, 1), b.r, a.c, 0, a.w, nd.bbar + a.r, -1.0));
    }
    R.copy(c);
    R.gemv(g);
  };
  for (int hh = 0; hh < maxh; ++hh) {
    std::vector<NR> v = nodes_at(hh);
    if (v.empty()) continue;
    merge(v);
    std::vector<CopyDesc> c1, c2;
    std::vector<GemvDesc> g1, g2, g3;
    std::vector<TrsvDesc> t1;
    for (auto& x : v) {
      HNode& nd = x.F->nd[x.t];
      double* bb = bbar_of(x);
      const int r = nd.r, nl = nd.nl;
      // c = Omega bbar
      c1.push_back(CV(bb, nd.dpermr + r, nd.ctop, nl));
      c1.push_back(CV(bb, nd.dpermr, nd.cbot, r));
      g1.push_back(GV(nd.Er, std::max(nl, 1), nl, r, 0, bb, nd.ctop, -1.0, 0, nd.dpermr));
      t1.push_back({nd.L, nullptr, nd.ctop, nl, std::max(nl, 1)});
      // chat = cbot - D21 y1 ; w = V1^T y1 (+ V^T [w_a; w_b])
      g2.push_back(GV(nd.WQ, std::max(r, 1), r, nl, 0, nd.ctop, nd.cbot, -1.0));
      g2.push_back(GV(nd.QV, nd.mr, nl, nd.c, 1, nd.ctop, nd.w, 1.0, 1));
      if (!nd.leaf()) {
        HNode& a = x.F->nd[nd.kid[0]];
        HNode& b = x.F->nd[nd.kid[1]];
        c2.push_back(CV(a.w, nullptr, nd.wab, a.c));
        c2.push_back(CV(b.w, nullptr, nd.wab + a.c, b.c));
        g3.push_back(GV(nd.Vd, std::max(nd.mc, 1), nd.mc, nd.c, 1, nd.wab, nd.w, 1.0));
      }
    }
    R.copy(c1);
    R.gemv(g1);
    R.trsv(t1, 4);
    R.gemv(g2);
    R.copy(c2);
    R.gemv(g3);
  }
  // top node k: LU solve of the merged block
  {
    std::vector<NR> v;
    for (auto& p : fs) v.push_back({p.first, p.first->k, p.second});
    merge(v);
    std::vector<TrsvDesc> t0;
    for (auto& x : v) t0.push_back({x.F->Dk, x.F->ipivk, bbar_of(x), x.F->mk, x.F->mk});
    R.trsv(t0, 0);
    R.trsv(t0, 1);
  }
  // down-sweep: xbar = Q [y1; y2] with y2 the parent's slice
  for (int hh = maxh - 1; hh >= 0; --hh) {
    std::vector<NR> v = nodes_at(hh);
    if (v.empty()) continue;
    std::vector<CopyDesc> c;
    std::vector<GemvDesc> g;
    for (auto& x : v) {
      HNode& nd = x.F->nd[x.t];
      HNode& p = x.F->nd[nd.parent];
      NR px{x.F, nd.parent, x.xv};
      double* pbuf = (nd.parent == x.F->k) ? bbar_of(px) : p.xbar;
      double* y2 = pbuf + ((p.kid[0] == x.t) ? 0 : x.F->nd[p.kid[0]].r);
      c.push_back(CV(nd.ctop, nullptr, nd.xin, nd.nl));
      c.push_back(CV(y2, nullptr, nd.xin + nd.nl, nd.r));
      double* out = nd.leaf() ? x.xv + nd.lo : nd.xbar;
      g.push_back(GV(nd.Q, nd.mr, nd.mr, nd.mr, 1, nd.xin, out, 1.0, 1));  // Q holds Qtilde^T
    }
    R.copy(c);
    R.gemv(g);
  }
}

// transposed ULV solve, F11^T lam = g in place on xv
void ulv_solve_t_rec(Rec& R, std::vector<std::pair<HFront*, double*>>& fs) {
  int maxh = 0;
  for (auto& p : fs) maxh = std::max(maxh, p.first->nd[p.first->k].height);
  auto nodes_at = [&](int hh) {
    std::vector<NR> v;
    for (auto& p : fs)
      for (int t = 0; t < (int)p.first->nd.size(); ++t)
        if (p.first->nd[t].height == hh && t != p.first->k && in_k(p.first, t)) v.push_back({p.first, t, p.second});
    return v;
  };
  auto gin = [](NR& x) -> double* {
    HNode& nd = x.F->nd[x.t];
    return nd.leaf() ? x.xv + nd.lo : nd.gbar;
  };
  auto stack = [&](std::vector<NR>& v) {
    std::vector<CopyDesc> c;
    for (auto& x : v) {
      HNode& nd = x.F->nd[x.t];
      if (nd.leaf()) continue;
      HNode& a = x.F->nd[nd.kid[0]];
      HNode& b = x.F->nd[nd.kid[1]];
      c.push_back(CV(a.gt + a.nl, nullptr, nd.gbar, a.r));
      c.push_back(CV(b.gt + b.nl, nullptr, nd.gbar + a.r, b.r));
    }
    R.copy(c);
  };
  for (int hh = 0; hh < maxh; ++hh) {
    std::vector<NR> v = nodes_at(hh);
    if (v.empty()) continue;
    stack(v);
    std::vector<GemvDesc> g;
    for (auto& x : v) {
      HNode& nd = x.F->nd[x.t];
      g.push_back(GV(nd.Q, nd.mr, nd.mr, nd.mr, 0, gin(x), nd.gt, 1.0, 1));  // Qtilde^T g
    }
    R.gemv(g);
  }
  {
    std::vector<NR> v;
    for (auto& p : fs) v.push_back({p.first, p.first->k, p.second});
    stack(v);
    std::vector<TrsvDesc> t0;
    for (auto& x : v) t0.push_back({x.F->Dk, x.F->ipivk, gin(x), x.F->mk, x.F->mk});
    R.trsv(t0, 2);
    R.trsv(t0, 3);
  }
  // down-sweep by parent height: children's coupling vectors h, then mu1 and
  // lam_child = Pi [mu2 - E^T mu1; mu1]
  for (int hp = maxh; hp >= 1; --hp) {
    std::vector<NR> parents;
    for (auto& p : fs)
      for (int t = 0; t < (int)p.first->nd.size(); ++t) {
        HNode& nd = p.first->nd[t];
        if (nd.height == hp && !nd.leaf() && in_k(p.first, t)) parents.push_back({p.first, t, p.second});
      }
    if (parents.empty()) continue;
    std::vector<GemvDesc> h1, h2, m1, m2, e1;
    std::vector<CopyDesc> c1, c2, c3;
    std::vector<TrsvDesc> tr;
    for (auto& x : parents) {
      HNode& nd = x.F->nd[x.t];
      HNode& a = x.F->nd[nd.kid[0]];
      HNode& b = x.F->nd[nd.kid[1]];
      double* lb = (x.t == x.F->k) ? gin(x) : nd.lbar;
      const double* mu_a = lb;
      const double* mu_b = lb + a.r;
      h1.push_back(GV(nd.B21, std::max(b.r, 1), b.r, a.c, 1, mu_b, a.hv, 1.0, 1));
      h1.push_back(GV(nd.B12, std::max(a.r, 1), a.r, b.c, 1, mu_a, b.hv, 1.0, 1));
      if (x.t != x.F->k) {
        h2.push_back(GV(nd.Vd, std::max(nd.mc, 1), a.c, nd.c, 0, nd.hv, a.hv, 1.0));
        h2.push_back(GV(nd.Vd + a.c, std::max(nd.mc, 1), b.c, nd.c, 0, nd.hv, b.hv, 1.0));
      }
      for (int s = 0; s < 2; ++s) {
        HNode& ch = s ? b : a;
        const double* mu2 = s ? mu_b : mu_a;
        const int nl = ch.nl, r = ch.r;
        c1.push_back(CV(ch.gt, nullptr, ch.tmp1, nl));
        m1.push_back(GV(ch.WQ, std::max(r, 1), r, nl, 1, mu2, ch.tmp1, -1.0));
        m2.push_back(GV(ch.QV, ch.mr, nl, ch.c, 0, ch.hv, ch.tmp1, -1.0));
        tr.push_back({ch.L, nullptr, ch.tmp1, nl, std::max(nl, 1)});
        c2.push_back(CV(mu2, nullptr, ch.tmpv, r));
        c2.push_back(CV(ch.tmp1, nullptr, ch.tmpv + r, nl));
        e1.push_back(GV(ch.Er, std::max(nl, 1), nl, r, 1, ch.tmp1, ch.tmpv, -1.0));
        double* out = ch.leaf() ? x.xv + ch.lo : ch.lbar;
        c3.push_back(CV(ch.tmpv, ch.diperm, out, ch.mr));
      }
    }
    R.gemv(h1);
    R.gemv(h2);
    R.copy(c1);
    R.gemv(m1);
    R.gemv(m2);
    R.trsv(tr, 5);
    R.copy(c2);
    R.gemv(e1);
    R.copy(c3);
  }
}

void alloc_solve_buffers(Handle& h) {
  auto D = [&](int64_t n) { return h.cur->get<double>((size_t)std::max<int64_t>(n, 1)); };
  for (auto& F : h.hf) {
    F.X = D(F.s);
    F.t1 = D(std::max(F.mk, F.n));
    F.t2 = D(std::max(F.mk, F.n));
    for (auto& nd : F.nd) {
      const int m = std::max(nd.mr, 1);
      nd.bbar = D(m); nd.ctop = D(m); nd.cbot = D(m); nd.w = D(std::max(nd.c, 1)); nd.wab = D(std::max(nd.mc, 1));
      nd.xin = D(m); nd.xbar = D(m); nd.gt = D(m); nd.gbar = D(m); nd.lbar = D(m); nd.hv = D(std::max(nd.c, 1));
      nd.tmp1 = D(m); nd.tmpv = D(m);
    }
  }
  // inverse row permutations of all nodes, one upload
  std::vector<int> all;
  std::vector<std::pair<HNode*, size_t>> at;
  for (auto& F : h.hf)
    for (auto& nd : F.nd)
      if (!nd.permr.empty()) {
        at.push_back({&nd, all.size()});
        size_t base = all.size();
        all.resize(base + nd.permr.size());
        for (size_t i = 0; i < nd.permr.size(); ++i) all[base + nd.permr[i]] = (int)i;
      }
  int* dall = upload(h, all);
  for (auto& pr : at) pr.first->diperm = dall + pr.second;
  for (auto& F : h.hf) {
    HNode& k = F.nd[F.k];
    if (!k.leaf()) k.bbar = D(F.mk), k.gbar = D(F.mk);
  }
}

}  // namespace

void build_solve_ops(Handle& h) {
  const Plan& P = h.P;
  alloc_solve_buffers(h);
  for (int tr = 0; tr < 2; ++tr)
    for (int sw = 0; sw < 2; ++sw) h.sops[tr][sw].clear();
  double* y = h.yws;
  Blob blob;
  for (int tr = 0; tr < 2; ++tr) {
    // forward sweep, bottom-up
    Rec R{h, h.sops[tr][0], blob};
    for (size_t lev = 0; lev < P.levels.size(); ++lev) {
      const auto& ids = P.levels[lev];
      std::vector<RhsDesc> rd;
      int mx = 0;
      for (int f : ids) {
        const FrontPlan& fp = P.fr[f];
        RhsDesc d{};
        d.y = y; d.w = h.fr[f].w; d.n = fp.n; d.s = fp.s; d.sep_lo = fp.lo; d.nkids = 0;
        for (size_t k = 0; k < fp.kids.size(); ++k) {
          if (P.fr[fp.kids[k]].u == 0) continue;
          d.wc[d.nkids] = h.fr[fp.kids[k]].w;
          d.inv[d.nkids] = h.fr[f].d_inv[k];
          d.nkids++;
        }
        rd.push_back(d);
        mx = std::max(mx, fp.n);
      }
      R.rhs(rd, mx);
      std::vector<TrsvDesc> t;
      std::vector<GemvDesc> g;
      std::vector<std::pair<HFront*, double*>> hs;
      for (int f : ids) {
        const FrontPlan& fp = P.fr[f];
        if (fp.hss) { hs.push_back({&h.hf[h.fr[f].hidx], y + fp.lo}); continue; }
        const double* F = h.fr[f].F;
        t.push_back({F, h.fr[f].ipiv, y + fp.lo, fp.s, fp.n});
        if (fp.u) {
          if (!tr) g.push_back(GV(F + fp.s, fp.n, fp.u, fp.s, 0, y + fp.lo, h.fr[f].w, -1.0));
          else g.push_back(GV(F + (int64_t)fp.s * fp.n, fp.n, fp.s, fp.u, 1, y + fp.lo, h.fr[f].w, -1.0));
        }
      }
      R.trsv(t, tr ? 2 : 0);
      R.gemv(g);
      if (!hs.empty()) {
        if (!tr) ulv_solve_rec(R, hs); else ulv_solve_t_rec(R, hs);
        // update part: w -= F21 z (or F12^T z) through the generators
        std::vector<GemvDesc> a, b, c;
        for (auto& p : hs) {
          HFront& F = *p.first;
          if (F.q < 0) continue;
          HNode& k = F.nd[F.k];
          HNode& q = F.nd[F.q];
          HNode& rt = F.nd[F.root];
          double* w = h.fr[F.f].w;
          if (!tr) {  // Ubig_q (B_qk (Vbig_k^T z))
            a.push_back(GV(k.Vbig, F.s, F.s, k.c, 1, p.second, F.t1, 1.0, 1));
            b.push_back(GV(rt.B21, std::max(q.r, 1), q.r, k.c, 0, F.t1, F.t2, 1.0, 1));
            c.push_back(GV(q.Ubig, F.u, F.u, q.r, 0, F.t2, w, -1.0));
          } else {    // Vbig_q (B_kq^T (Ubig_k^T z))
            a.push_back(GV(k.Ubig, F.s, F.s, k.r, 1, p.second, F.t1, 1.0, 1));
            b.push_back(GV(rt.B12, std::max(k.r, 1), k.r, q.c, 1, F.t1, F.t2, 1.0, 1));
            c.push_back(GV(q.Vbig, F.u, F.u, q.c, 0, F.t2, w, -1.0));
          }
        }
        R.gemv(a); R.gemv(b); R.gemv(c);
      }
    }
    // backward sweep, top-down
    Rec B{h, h.sops[tr][1], blob};
    for (int lev = (int)P.levels.size() - 1; lev >= 0; --lev) {
      const auto& ids = P.levels[lev];
      std::vector<GemvDesc> g;
      std::vector<TrsvDesc> t;
      std::vector<std::pair<HFront*, double*>> hs;
      std::vector<GemvDesc> a, b, c;
      for (int f : ids) {
        const FrontPlan& fp = P.fr[f];
        if (fp.hss) {
          HFront& F = h.hf[h.fr[f].hidx];
          if (F.q < 0) continue;
          hs.push_back({&F, F.X});
          HNode& k = F.nd[F.k];
          HNode& q = F.nd[F.q];
          HNode& rt = F.nd[F.root];
          const int* um = h.fr[f].d_upd;
          if (!tr) {  // X = Ubig_k (B_kq (Vbig_q^T x_upd))
            a.push_back(GV(q.Vbig, F.u, F.u, q.c, 1, y, F.t1, 1.0, 1, um));
            b.push_back(GV(rt.B12, std::max(k.r, 1), k.r, q.c, 0, F.t1, F.t2, 1.0, 1));
            c.push_back(GV(k.Ubig, F.s, F.s, k.r, 0, F.t2, F.X, 1.0, 1));
          } else {    // X = Vbig_k (B_qk^T (Ubig_q^T x_upd))
            a.push_back(GV(q.Ubig, F.u, F.u, q.r, 1, y, F.t1, 1.0, 1, um));
            b.push_back(GV(rt.B21, std::max(q.r, 1), q.r, k.c, 1, F.t1, F.t2, 1.0, 1));
            c.push_back(GV(k.Vbig, F.s, F.s, k.c, 0, F.t2, F.X, 1.0, 1));
          }
          continue;
        }
        const double* F = h.fr[f].F;
        if (fp.u) {
          if (!tr) g.push_back(GV(F + (int64_t)fp.s * fp.n, fp.n, fp.s, fp.u, 0, y, y + fp.lo, -1.0, 0, h.fr[f].d_upd));
          else g.push_back(GV(F + fp.s, fp.n, fp.u, fp.s, 1, y, y + fp.lo, -1.0, 0, h.fr[f].d_upd));
        }
        t.push_back({F, h.fr[f].ipiv, y + fp.lo, fp.s, fp.n});
      }
      B.gemv(g);
      B.trsv(t, tr ? 3 : 1);
      if (!hs.empty()) {
        B.gemv(a); B.gemv(b); B.gemv(c);
        if (!tr) ulv_solve_rec(B, hs); else ulv_solve_t_rec(B, hs);
        std::vector<CopyDesc> cp;
        for (auto& p : hs) cp.push_back(CV(p.first->X, nullptr, y + P.fr[p.first->f].lo, p.first->s, 1, -1.0));
        B.copy(cp);
      }
    }
  }
  char* dev = h.cur->get<char>(std::max<size_t>(blob.bytes.size(), 1));
  if (!blob.bytes.empty())
    HIP_CHECK(hipMemcpyAsync(dev, blob.bytes.data(), blob.bytes.size(), hipMemcpyHostToDevice, h.st));
  HIP_CHECK(hipStreamSynchronize(h.st));  // the blob is pageable host memory
  for (int tr = 0; tr < 2; ++tr)
    for (int sw = 0; sw < 2; ++sw)
      for (Op& o : h.sops[tr][sw]) {
        o.d = dev + reinterpret_cast<size_t>(o.d);
        if (o.ws) o.ws = reinterpret_cast<int*>(dev + reinterpret_cast<size_t>(o.ws));
      }
}

void run_ops(Handle& h, const std::vector<Op>& ops) {
  for (const Op& o : ops) {
    switch (o.kind) {
      case OP_GEMV: launch_gemv((const GemvDesc*)o.d, o.n, (int)o.p0, h.st); break;
      case OP_COPY: launch_copy(device_batch<CopyDesc, 32>((const CopyDesc*)o.d), o.n, o.p0, 0, h.st); break;
      case OP_TRSV:
        if (o.ws)
          launch_trsv_multi((const TrsvDesc*)o.d, o.n, (int)(o.p0 % 16), (int)(o.p0 / 16), o.ws, h.werr_d, h.st);
        else
          launch_trsv((const TrsvDesc*)o.d, o.n, (int)(o.p0 % 16), (int)(o.p0 / 16), h.st);
        break;
      case OP_RHS: launch_rhs_gather((const RhsDesc*)o.d, o.n, (int)o.p0, h.st); break;
    }
  }
}

// forward and backward sweeps on the handle's work vector, replayed as one
// HIP graph when enabled (captured on first use after each factorization:
// the sweeps only launch kernels on descriptors already on the device)
void sweeps(Handle& h, int trans, bool graph) {
  if (!h.o.use_graph || !graph) {
    run_ops(h, h.sops[trans][0]);
    run_ops(h, h.sops[trans][1]);
    return;
  }
  if (!h.gexec[trans]) {
    if (!h.gst) HIP_CHECK(hipStreamCreateWithFlags(&h.gst, hipStreamNonBlocking));
    hipStream_t user = h.st;
    h.st = h.gst;
    hipGraph_t g = nullptr;
    HIP_CHECK(hipStreamBeginCapture(h.gst, hipStreamCaptureModeThreadLocal));
    try {
      run_ops(h, h.sops[trans][0]);
      run_ops(h, h.sops[trans][1]);
    } catch (...) {
      (void)hipStreamEndCapture(h.gst, &g);
      if (g) (void)hipGraphDestroy(g);
      h.st = user;
      throw;
    }
    h.st = user;
    HIP_CHECK(hipStreamEndCapture(h.gst, &g));
    hipError_t e = hipGraphInstantiate(&h.gexec[trans], g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    HIP_CHECK(e);
  }
  HIP_CHECK(hipGraphLaunch(h.gexec[trans], h.st));
}

void apply_inverse(Handle& h, int trans, const double* x, double* yout, bool graph) {
  const int n = h.P.n;
  launch_gather(h.yws, x, h.d_perm, n, h.st);
  sweeps(h, trans, graph);
  launch_gather(yout, h.yws, h.d_iperm, n, h.st);
}

void spmv(Handle& h, int trans, const double* x, double* y, double alpha, double beta) {
  if (!trans) launch_spmv(h.d_rowptr, h.d_colind, h.d_val, nullptr, x, y, h.P.n, alpha, beta, h.st);
  else launch_spmv(h.d_trowptr, h.d_tcolind, h.d_val, h.d_tvidx, x, y, h.P.n, alpha, beta, h.st);
}

double dnrm2(Handle& h, const double* x, int n) {
  launch_dot(x, x, n, h.d_part, h.d_scal, 1, h.st);
  double r = 0;
  HIP_CHECK(hipMemcpyAsync(&r, h.d_scal, sizeof(double), hipMemcpyDeviceToHost, h.st));
  HIP_CHECK(hipStreamSynchronize(h.st));
  h.stager.sync();
  return r;
}

}  // namespace hssmf
