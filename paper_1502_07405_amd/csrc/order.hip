// Algebraic front end on the host (Sec. 3.1, Sec. 4.2): static scaling and
// column permutation of A for stability (a maximum-product matching with
// the matching's dual variables as scalings, the MC64 approach of Duff and
// Koster), and a fill-reducing nested dissection of the graph of A + A^T
// whose separators are then ordered for HSS compression by recursive
// bisection of the separator graph enriched with length-two connections.
// The nested dissection here splits a vertex set at the middle level of a
// breadth-first level structure from a pseudo-peripheral vertex (George's
// level-structure dissection) in place of a graph partitioning library.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <functional>
#include <limits>
#include <queue>
#include <vector>

#include "common.hpp"

namespace hssmf {
namespace {

// the pattern of A + A^T without the diagonal, as adjacency lists
struct Graph {
  int n = 0;
  std::vector<int> ptr, adj;
  int deg(int v) const { return ptr[v + 1] - ptr[v]; }
};

Graph symmetric_graph(const hssmf_csr& A) {
  const int n = A.n;
  std::vector<std::vector<int>> nb(n);
  for (int i = 0; i < n; ++i)
    for (int64_t e = A.rowptr[i]; e < A.rowptr[i + 1]; ++e) {
      const int j = A.colind[e];
      if (j == i) continue;
      nb[i].push_back(j);
      nb[j].push_back(i);
    }
  Graph g;
  g.n = n;
  g.ptr.assign(n + 1, 0);
  for (int i = 0; i < n; ++i) {
    std::sort(nb[i].begin(), nb[i].end());
    nb[i].erase(std::unique(nb[i].begin(), nb[i].end()), nb[i].end());
    g.ptr[i + 1] = g.ptr[i] + (int)nb[i].size();
  }
  g.adj.reserve(g.ptr[n]);
  for (int i = 0; i < n; ++i) g.adj.insert(g.adj.end(), nb[i].begin(), nb[i].end());
  return g;
}

bool csr_ok(const hssmf_csr* A) {
  if (!A || A->n < 1 || !A->rowptr || !A->colind || A->mem != HSSMF_MEM_HOST) return false;
  if (A->rowptr[0] != 0) return false;
  for (int i = 0; i < A->n; ++i) {
    if (A->rowptr[i + 1] < A->rowptr[i]) return false;
    for (int64_t e = A->rowptr[i]; e < A->rowptr[i + 1]; ++e)
      if (A->colind[e] < 0 || A->colind[e] >= A->n) return false;
  }
  return true;
}

// Breadth-first search inside the vertices with in[v] == tag, from root;
// lev[v] receives the level, the return value the vertices in visiting order
// (one component)
std::vector<int> bfs(const Graph& g, const std::vector<int>& in, int tag, int root, std::vector<int>& lev) {
  std::vector<int> q{root};
  lev[root] = 0;
  for (size_t h = 0; h < q.size(); ++h) {
    const int v = q[h];
    for (int e = g.ptr[v]; e < g.ptr[v + 1]; ++e) {
      const int w = g.adj[e];
      if (in[w] == tag && lev[w] < 0) {
        lev[w] = lev[v] + 1;
        q.push_back(w);
      }
    }
  }
  return q;
}

// a pseudo-peripheral vertex of the component of start: repeat a search
// from a vertex of smallest degree on the last level while the number of
// levels grows
int peripheral(const Graph& g, const std::vector<int>& in, int tag, int start, std::vector<int>& lev) {
  int r = start, ecc = -1;
  for (int it = 0; it < 8; ++it) {
    std::vector<int> q = bfs(g, in, tag, r, lev);
    const int e = lev[q.back()];
    int best = q.back();
    for (int v : q)
      if (lev[v] == e && g.deg(v) < g.deg(best)) best = v;
    for (int v : q) lev[v] = -1;
    if (e <= ecc) break;
    ecc = e;
    r = best;
  }
  return r;
}

struct NDBuilder {
  const Graph& g;
  int leaf, sep_leaf;
  std::vector<int> in, lev;   // membership tags, levels (-1 = unset)
  std::vector<int> loc;       // separator-local index of a vertex (-1 = none)
  int tag = 0;
  std::vector<int> perm, sep_ptr{0}, parent;

  NDBuilder(const Graph& gr, int lf, int sl)
      : g(gr), leaf(lf), sep_leaf(sl), in(gr.n, 0), lev(gr.n, -1), loc(gr.n, -1) {}

  // a new front owning the vertices of sep (ordered for HSS compression
  // when it is long), children a and b (-1: none); returns its id
  int emit(std::vector<int> sep, int a, int b) {
    if ((int)sep.size() > sep_leaf) sep = order_separator(sep);
    const int f = (int)parent.size();
    perm.insert(perm.end(), sep.begin(), sep.end());
    sep_ptr.push_back((int)perm.size());
    parent.push_back(-1);
    if (a >= 0) parent[a] = f;
    if (b >= 0) parent[b] = f;
    return f;
  }

  // Sec. 4.2: recursive bisection of the separator graph, with an edge
  // between two separator vertices when they are adjacent or share a
  // neighbour; each half is the first (or last) ceil(n / 2) vertices of a
  // breadth-first order from a pseudo-peripheral vertex, so that the
  // halves are the leaves' index ranges of the front's HSS tree
  std::vector<int> order_separator(const std::vector<int>& sep) {
    const int m = (int)sep.size();
    for (int i = 0; i < m; ++i) loc[sep[i]] = i;
    Graph s;
    s.n = m;
    s.ptr.assign(m + 1, 0);
    std::vector<std::vector<int>> nb(m);
    for (int i = 0; i < m; ++i) {
      const int u = sep[i];
      for (int e = g.ptr[u]; e < g.ptr[u + 1]; ++e) {
        const int x = g.adj[e];
        if (loc[x] >= 0) nb[i].push_back(loc[x]);
        for (int f = g.ptr[x]; f < g.ptr[x + 1]; ++f) {
          const int w = g.adj[f];
          if (loc[w] >= 0 && w != u) nb[i].push_back(loc[w]);
        }
      }
      std::sort(nb[i].begin(), nb[i].end());
      nb[i].erase(std::unique(nb[i].begin(), nb[i].end()), nb[i].end());
      s.ptr[i + 1] = s.ptr[i] + (int)nb[i].size();
    }
    for (int i = 0; i < m; ++i) s.adj.insert(s.adj.end(), nb[i].begin(), nb[i].end());
    std::vector<int> sin(m, 0), slev(m, -1), out;
    out.reserve(m);
    int stag = 0;
    std::vector<int> all(m);
    for (int i = 0; i < m; ++i) all[i] = i;
    std::function<void(const std::vector<int>&)> rec = [&](const std::vector<int>& part) {
      if ((int)part.size() <= sep_leaf) {
        out.insert(out.end(), part.begin(), part.end());
        return;
      }
      ++stag;
      for (int v : part) sin[v] = stag;
      // breadth-first order over every component of the part
      std::vector<int> ord;
      for (int v0 : part) {
        if (slev[v0] >= 0) continue;
        const int r = peripheral(s, sin, stag, v0, slev);
        std::vector<int> q = bfs(s, sin, stag, r, slev);
        ord.insert(ord.end(), q.begin(), q.end());
      }
      for (int v : part) slev[v] = -1;
      const size_t h = (ord.size() + 1) / 2;
      rec(std::vector<int>(ord.begin(), ord.begin() + h));
      rec(std::vector<int>(ord.begin() + h, ord.end()));
    };
    rec(all);
    std::vector<int> res(m);
    for (int i = 0; i < m; ++i) res[i] = sep[out[i]];
    for (int i = 0; i < m; ++i) loc[sep[i]] = -1;
    return res;
  }

  // nested dissection of the vertex set V: fronts of the two parts in
  // postorder, then the separator's front
  int dissect(const std::vector<int>& V) {
    if ((int)V.size() <= leaf) return emit(V, -1, -1);
    ++tag;
    const int t = tag;
    for (int v : V) in[v] = t;
    int start = V[0];
    for (int v : V)
      if (g.deg(v) < g.deg(start)) start = v;
    const int r = peripheral(g, in, t, start, lev);
    std::vector<int> q = bfs(g, in, t, r, lev);
    if (q.size() < V.size()) {
      // V is disconnected: one vertex of the searched component (the last
      // reached) separates the rest of that component from the others
      std::vector<int> rest;
      for (int v : V)
        if (lev[v] < 0) rest.push_back(v);
      for (int v : q) lev[v] = -1;
      const int x = q.back();
      q.pop_back();
      const int a = q.empty() ? -1 : dissect(q);
      const int b = dissect(rest);
      return emit(std::vector<int>{x}, a, b);
    }
    const int nl = lev[q.back()] + 1;
    if (nl < 3) {   // no level can separate: one front
      for (int v : q) lev[v] = -1;
      return emit(V, -1, -1);
    }
    std::vector<int> cnt(nl, 0);
    for (int v : q) cnt[lev[v]]++;
    // the middle level: the first whose cumulative count reaches half of V
    int L = 0, cum = 0;
    while (L < nl && cum + cnt[L] < (int)V.size() / 2) cum += cnt[L++];
    L = std::max(1, std::min(L, nl - 2));
    std::vector<int> A, S, B;
    for (int v : q) (lev[v] < L ? A : lev[v] == L ? S : B).push_back(v);
    // separator vertices without a neighbour on the far side join the near side
    std::vector<int> S2;
    for (int v : S) {
      bool far = false;
      for (int e = g.ptr[v]; e < g.ptr[v + 1] && !far; ++e) {
        const int w = g.adj[e];
        far = in[w] == t && lev[w] > L;
      }
      (far ? S2 : A).push_back(v);
    }
    for (int v : q) lev[v] = -1;
    const int a = dissect(A);
    const int b = dissect(B);
    return emit(S2, a, b);
  }
};

}  // namespace
}  // namespace hssmf

extern "C" int hssmf_nested_dissection(const hssmf_csr* A, int32_t leaf_size, int32_t sep_leaf, int32_t* perm,
                                       int32_t* sep_ptr, int32_t* parent, int32_t* nfront) {
  using namespace hssmf;
  if (!csr_ok(A) || leaf_size < 1 || sep_leaf < 1 || !perm || !sep_ptr || !parent || !nfront) return HSSMF_EINVAL;
  try {
    const Graph g = symmetric_graph(*A);
    NDBuilder b(g, leaf_size, sep_leaf);
    std::vector<int> all(A->n);
    for (int i = 0; i < A->n; ++i) all[i] = i;
    b.dissect(all);
    // empty separators (a front that only joins two subtrees) are folded
    // into their parent: the multifrontal plan needs every front to own
    // at least one index
    const int nf = (int)b.parent.size();
    std::vector<int> keep(nf, 1), id(nf, -1);
    for (int f = 0; f < nf; ++f) keep[f] = b.sep_ptr[f + 1] > b.sep_ptr[f];
    REQUIRE(keep[nf - 1], HSSMF_EINVAL, "nested dissection: the root owns no index");
    int k = 0;
    for (int f = 0; f < nf; ++f)
      if (keep[f]) id[f] = k++;
    sep_ptr[0] = 0;
    for (int f = 0, o = 0; f < nf; ++f) {
      if (!keep[f]) continue;
      int p = b.parent[f];
      while (p >= 0 && !keep[p]) p = b.parent[p];
      parent[id[f]] = p >= 0 ? id[p] : -1;
      o += b.sep_ptr[f + 1] - b.sep_ptr[f];
      sep_ptr[id[f] + 1] = o;
    }
    std::memcpy(perm, b.perm.data(), sizeof(int32_t) * A->n);
    *nfront = k;
    return HSSMF_OK;
  } catch (const Error& e) {
    return e.code;
  } catch (...) {
    return HSSMF_EINVAL;
  }
}

extern "C" int hssmf_static_pivoting(const hssmf_csr* A, int32_t* colperm, double* row_scale, double* col_scale) {
  using namespace hssmf;
  if (!csr_ok(A) || !A->val || !colperm || !row_scale || !col_scale) return HSSMF_EINVAL;
  const int n = A->n;
  // columns of A (nonzero entries only), costs c_ij = log max_k |a_kj| - log |a_ij| >= 0
  std::vector<int64_t> cp(n + 1, 0);
  for (int64_t e = 0; e < A->rowptr[n]; ++e)
    if (A->val[e] != 0.0) cp[A->colind[e] + 1]++;
  for (int j = 0; j < n; ++j) cp[j + 1] += cp[j];
  std::vector<int> ri(cp[n]);
  std::vector<double> cost(cp[n]);
  {
    std::vector<int64_t> fill(cp.begin(), cp.end() - 1);
    for (int i = 0; i < n; ++i)
      for (int64_t e = A->rowptr[i]; e < A->rowptr[i + 1]; ++e) {
        if (A->val[e] == 0.0) continue;
        const int64_t p = fill[A->colind[e]]++;
        ri[p] = i;
        cost[p] = std::log(std::fabs(A->val[e]));
      }
  }
  std::vector<double> cmax(n, -std::numeric_limits<double>::infinity());
  for (int j = 0; j < n; ++j) {
    if (cp[j] == cp[j + 1]) return HSSMF_ESINGULAR;   // an empty column
    for (int64_t p = cp[j]; p < cp[j + 1]; ++p) cmax[j] = std::max(cmax[j], cost[p]);
    for (int64_t p = cp[j]; p < cp[j + 1]; ++p) cost[p] = cmax[j] - cost[p];
  }
  // dual variables: c_ij - u_i - v_j >= 0, equality on the matching
  const double inf = std::numeric_limits<double>::infinity();
  std::vector<double> u(n, inf), v(n, 0.0);
  for (int j = 0; j < n; ++j)
    for (int64_t p = cp[j]; p < cp[j + 1]; ++p) u[ri[p]] = std::min(u[ri[p]], cost[p]);
  for (int i = 0; i < n; ++i)
    if (u[i] == inf) return HSSMF_ESINGULAR;          // an empty row
  std::vector<int> mrow(n, -1), mcol(n, -1), pred(n, -1);
  std::vector<double> dist(n, inf), dcol(n, inf);
  std::vector<char> done(n, 0);
  using QE = std::pair<double, int>;
  // shortest augmenting paths (Dijkstra on the reduced costs), one free
  // column at a time
  for (int j0 = 0; j0 < n; ++j0) {
    std::priority_queue<QE, std::vector<QE>, std::greater<QE>> pq;
    std::vector<int> touched, srows, scols{j0};
    dcol[j0] = 0.0;
    for (int64_t p = cp[j0]; p < cp[j0 + 1]; ++p) {
      const int i = ri[p];
      const double d = cost[p] - u[i] - v[j0];
      if (d < dist[i]) {
        if (dist[i] == inf) touched.push_back(i);
        dist[i] = d;
        pred[i] = j0;
        pq.push({d, i});
      }
    }
    int ifree = -1;
    double D = inf;
    while (!pq.empty()) {
      const auto [d, i] = pq.top();
      pq.pop();
      if (done[i] || d > dist[i]) continue;
      done[i] = 1;
      srows.push_back(i);
      if (mrow[i] < 0) {
        ifree = i;
        D = d;
        break;
      }
      const int j = mrow[i];
      dcol[j] = d;
      scols.push_back(j);
      for (int64_t p = cp[j]; p < cp[j + 1]; ++p) {
        const int i2 = ri[p];
        if (done[i2]) continue;
        const double nd = d + (cost[p] - u[i2] - v[j]);
        if (nd < dist[i2]) {
          if (dist[i2] == inf) touched.push_back(i2);
          dist[i2] = nd;
          pred[i2] = j;
          pq.push({nd, i2});
        }
      }
    }
    if (ifree < 0) return HSSMF_ESINGULAR;            // no perfect matching
    for (int i : srows) u[i] -= D - dist[i];
    for (int j : scols) v[j] += D - dcol[j];
    for (int i = ifree;;) {
      const int j = pred[i];
      const int prev = mcol[j];
      mcol[j] = i;
      mrow[i] = j;
      if (j == j0) break;
      i = prev;
    }
    for (int i : touched) {
      dist[i] = inf;
      done[i] = 0;
    }
    for (int j : scols) dcol[j] = inf;
  }
  for (int i = 0; i < n; ++i) {
    colperm[i] = mrow[i];
    row_scale[i] = std::exp(u[i]);
  }
  for (int j = 0; j < n; ++j) col_scale[j] = std::exp(v[j] - cmax[j]);
  return HSSMF_OK;
}
