// Host planning: validation of the CSR matrix and the ordering, the
// permuted structure, update index sets of the fronts (symbolic
// factorization, Sec. 5.4), elimination-tree heights, child-to-parent maps,
// and the device arena / descriptor staging.
#include <algorithm>
#include <cstring>
#include <mutex>
#include <numeric>

#include "solver.hpp"

namespace hssmf {

// ------------------------------------------------------------ arena --------
namespace {
std::mutex g_cache_mu;
std::vector<std::pair<char*, size_t>> g_cache;  // released chunks for reuse
size_t g_cached = 0;
constexpr size_t kCacheCap = size_t(64) << 30;  // keep at most 64 GB of released chunks

void cache_put(char* p, size_t sz) {
  g_cache.push_back({p, sz});
  g_cached += sz;
  // bounded cache: give the largest chunks back to the runtime first
  while (g_cached > kCacheCap && !g_cache.empty()) {
    size_t big = 0;
    for (size_t i = 1; i < g_cache.size(); ++i)
      if (g_cache[i].second > g_cache[big].second) big = i;
    (void)hipFree(g_cache[big].first);
    g_cached -= g_cache[big].second;
    g_cache.erase(g_cache.begin() + big);
  }
}
}  // namespace

void* Arena::alloc(size_t bytes, size_t align) {
  if (bytes == 0) bytes = align;
  size_t need = (bytes + align - 1) / align * align;
  if (chunks_.empty() || off_ + need > chunks_.back().size) {
    size_t sz = std::max<size_t>(need, size_t(256) << 20);
    char* p = nullptr;
    {
      // best fit among the cached chunks
      std::lock_guard<std::mutex> g(g_cache_mu);
      size_t bi = g_cache.size();
      for (size_t i = 0; i < g_cache.size(); ++i)
        if (g_cache[i].second >= sz && (bi == g_cache.size() || g_cache[i].second < g_cache[bi].second)) bi = i;
      if (bi < g_cache.size() && g_cache[bi].second <= 4 * sz) {
        p = g_cache[bi].first;
        sz = g_cache[bi].second;
        g_cached -= sz;
        g_cache.erase(g_cache.begin() + bi);
      }
    }
    if (!p) {
      hipError_t e = hipMalloc(&p, sz);
      if (e != hipSuccess) {
        (void)hipGetLastError();
        // return the cache to the runtime and try once more
        {
          std::lock_guard<std::mutex> g(g_cache_mu);
          for (auto& c : g_cache) (void)hipFree(c.first);
          g_cache.clear();
          g_cached = 0;
        }
        e = hipMalloc(&p, sz);
        if (e != hipSuccess) {
          (void)hipGetLastError();
          throw Error(HSSMF_ENOMEM, "device allocation of " + std::to_string(sz) + " bytes failed");
        }
      }
    }
    chunks_.push_back({p, sz});
    off_ = 0;
  }
  char* r = chunks_.back().p + off_;
  off_ += need;
  used_ += need;
  peak_ = std::max(peak_, used_);
  return r;
}

void Arena::reset(const Mark& m) {
  // chunks allocated after the mark go back to the cache
  std::lock_guard<std::mutex> g(g_cache_mu);
  while (chunks_.size() > m.chunk + 1) {
    cache_put(chunks_.back().p, chunks_.back().size);
    chunks_.pop_back();
  }
  off_ = m.off;
  used_ = m.used;
}

void arena_trim_cache() {
  std::lock_guard<std::mutex> g(g_cache_mu);
  for (auto& c : g_cache) (void)hipFree(c.first);
  g_cache.clear();
  g_cached = 0;
}

void Arena::release() {
  std::lock_guard<std::mutex> g(g_cache_mu);
  for (auto& c : chunks_) cache_put(c.p, c.size);
  chunks_.clear();
  off_ = used_ = 0;
}

// ----------------------------------------------------------- stager --------
void Stager::init(size_t bytes) {
  cap_ = bytes;
  HIP_CHECK(hipHostMalloc((void**)&host_, bytes, hipHostMallocDefault));
  HIP_CHECK(hipMalloc((void**)&dev_, bytes));
  ws_elems = size_t(32) << 20;  // 256 MB of doubles
  HIP_CHECK(hipMalloc((void**)&ws, ws_elems * sizeof(double)));
}

Stager::~Stager() {
  if (host_) (void)hipHostFree(host_);
  if (dev_) (void)hipFree(dev_);
  if (ws) (void)hipFree(ws);
}

void* Stager::put(const void* src, size_t bytes, hipStream_t s) {
  size_t need = (bytes + 255) / 256 * 256;
  REQUIRE(need <= cap_, HSSMF_ENOMEM, "descriptor staging buffer too small");
  if (off_ + need > cap_) {
    HIP_CHECK(hipStreamSynchronize(s));
    off_ = 0;
  }
  std::memcpy(host_ + off_, src, bytes);
  HIP_CHECK(hipMemcpyAsync(dev_ + off_, host_ + off_, bytes, hipMemcpyHostToDevice, s));
  ++n_put;
  void* r = dev_ + off_;
  off_ += need;
  return r;
}

void Stager::put_to(void* dst, const void* src, size_t bytes, hipStream_t s) {
  size_t need = (bytes + 255) / 256 * 256;
  if (need > cap_) {
    HIP_CHECK(hipStreamSynchronize(s));
    HIP_CHECK(hipMemcpy(dst, src, bytes, hipMemcpyHostToDevice));
    return;
  }
  if (off_ + need > cap_) {
    HIP_CHECK(hipStreamSynchronize(s));
    off_ = 0;
  }
  std::memcpy(host_ + off_, src, bytes);
  HIP_CHECK(hipMemcpyAsync(dst, host_ + off_, bytes, hipMemcpyHostToDevice, s));
  ++n_put_to;
  off_ += need;
}

// ------------------------------------------------------------- plan --------
void build_plan(const hssmf_csr* A, const hssmf_ordering* ord, const hssmf_opts* o, Plan& P) {
  REQUIRE(A && ord && o, HSSMF_EINVAL, "null argument");
  REQUIRE(A->n >= 0 && A->rowptr && (A->n == 0 || (A->colind && A->val)), HSSMF_EINVAL, "bad CSR header");
  const int n = A->n;
  P.n = n;
  REQUIRE(A->rowptr[0] == 0, HSSMF_EINVAL, "rowptr[0] != 0");
  for (int i = 0; i < n; ++i) REQUIRE(A->rowptr[i + 1] >= A->rowptr[i], HSSMF_EINVAL, "rowptr not monotone");
  P.nnz = A->rowptr[n];
  for (int64_t e = 0; e < P.nnz; ++e)
    REQUIRE(A->colind[e] >= 0 && A->colind[e] < n, HSSMF_EINVAL, "column index out of range");
  // ordering
  REQUIRE(ord->perm && ord->sep_ptr && ord->parent && ord->nfront >= (n > 0 ? 1 : 0), HSSMF_EINVAL,
          "bad ordering header");
  P.perm.assign(ord->perm, ord->perm + n);
  P.iperm.assign(n, -1);
  for (int i = 0; i < n; ++i) {
    int v = P.perm[i];
    REQUIRE(v >= 0 && v < n && P.iperm[v] < 0, HSSMF_EINVAL, "perm is not a permutation");
    P.iperm[v] = i;
  }
  const int nf = ord->nfront;
  P.nfront = nf;
  REQUIRE(ord->sep_ptr[0] == 0 && ord->sep_ptr[nf] == n, HSSMF_EINVAL, "sep_ptr must span [0, n)");
  for (int f = 0; f < nf; ++f) {
    REQUIRE(ord->sep_ptr[f + 1] >= ord->sep_ptr[f], HSSMF_EINVAL, "sep_ptr not monotone");
    int p = ord->parent[f];
    REQUIRE(p == -1 || (p > f && p < nf), HSSMF_EINVAL, "parent must follow its child (postorder)");
  }
  for (int i = 0; i < n; ++i) {
    int64_t b = A->rowptr[P.perm[i]], e = A->rowptr[P.perm[i] + 1];
    for (int64_t x = b; x < e; ++x)
      for (int64_t y = x + 1; y < e; ++y)
        if (e - b < 64) REQUIRE(A->colind[x] != A->colind[y], HSSMF_EINVAL, "duplicate entry in a row");
  }
  // permuted CSR with sorted columns
  P.prow.assign(n + 1, 0);
  P.pcol.resize(P.nnz);
  P.pvidx.resize(P.nnz);
  {
    std::vector<std::pair<int, int64_t>> tmp;
    int64_t pos = 0;
    for (int i = 0; i < n; ++i) {
      int old = P.perm[i];
      tmp.clear();
      for (int64_t e = A->rowptr[old]; e < A->rowptr[old + 1]; ++e) tmp.push_back({P.iperm[A->colind[e]], e});
      std::sort(tmp.begin(), tmp.end());
      for (auto& t : tmp) {
        P.pcol[pos] = t.first;
        P.pvidx[pos] = t.second;
        ++pos;
      }
      P.prow[i + 1] = pos;
    }
  }
  // transpose structure
  P.trow.assign(n + 1, 0);
  for (int64_t e = 0; e < P.nnz; ++e) P.trow[P.pcol[e] + 1]++;
  for (int i = 0; i < n; ++i) P.trow[i + 1] += P.trow[i];
  P.tcol.resize(P.nnz);
  P.tvidx.resize(P.nnz);
  {
    std::vector<int64_t> fill(P.trow.begin(), P.trow.end() - 1);
    for (int i = 0; i < n; ++i)
      for (int64_t e = P.prow[i]; e < P.prow[i + 1]; ++e) {
        int64_t p = fill[P.pcol[e]]++;
        P.tcol[p] = i;
        P.tvidx[p] = P.pvidx[e];
      }
  }
  // fronts
  P.fr.resize(nf);
  std::vector<int> front_of(n);
  for (int f = 0; f < nf; ++f) {
    FrontPlan& F = P.fr[f];
    F.id = f;
    F.lo = ord->sep_ptr[f];
    F.hi = ord->sep_ptr[f + 1];
    F.s = F.hi - F.lo;
    F.parent = ord->parent[f];
    for (int i = F.lo; i < F.hi; ++i) front_of[i] = f;
  }
  for (int f = 0; f < nf; ++f)
    if (P.fr[f].parent >= 0) P.fr[P.fr[f].parent].kids.push_back(f);
  // separator property: a coupling joins a front with itself or an ancestor
  auto is_anc = [&](int a, int d) {  // is a an ancestor of d (or equal)
    while (d >= 0 && d < a) d = P.fr[d].parent;
    return d == a;
  };
  for (int i = 0; i < n; ++i)
    for (int64_t e = P.prow[i]; e < P.prow[i + 1]; ++e) {
      int fi = front_of[i], fj = front_of[P.pcol[e]];
      if (fi == fj) continue;
      REQUIRE(fi < fj ? is_anc(fj, fi) : is_anc(fi, fj), HSSMF_EINVAL,
              "ordering violates the separator property");
    }
  // update sets (children's sets plus direct couplings beyond the separator)
  std::vector<int> mark(n, -1);
  for (int f = 0; f < nf; ++f) {
    FrontPlan& F = P.fr[f];
    std::vector<int>& U = F.upd;
    auto add = [&](int j) {
      if (j >= F.hi && mark[j] != f) {
        mark[j] = f;
        U.push_back(j);
      }
    };
    for (int i = F.lo; i < F.hi; ++i) {
      for (int64_t e = P.prow[i]; e < P.prow[i + 1]; ++e) add(P.pcol[e]);
      for (int64_t e = P.trow[i]; e < P.trow[i + 1]; ++e) add(P.tcol[e]);
    }
    for (int c : F.kids)
      for (int j : P.fr[c].upd) add(j);
    std::sort(U.begin(), U.end());
    F.u = (int)U.size();
    F.n = F.s + F.u;
    F.hss = F.s >= o->min_sep_hss;
    int h = 0;
    for (int c : F.kids) h = std::max(h, P.fr[c].height + 1);
    F.height = h;
    if (F.kids.size() > 2)
      throw Error(HSSMF_EINVAL, "separator tree must be binary (a front has more than two children)");
  }
  for (int f = 0; f < nf; ++f) {
    FrontPlan& F = P.fr[f];
    for (int c : F.kids) {
      const FrontPlan& C = P.fr[c];
      std::vector<int> m(C.u);
      for (int t = 0; t < C.u; ++t) {
        int j = C.upd[t];
        if (j < F.hi) {
          REQUIRE(j >= F.lo, HSSMF_EINVAL, "child update index outside the parent front");
          m[t] = j - F.lo;
        } else {
          auto it = std::lower_bound(F.upd.begin(), F.upd.end(), j);
          REQUIRE(it != F.upd.end() && *it == j, HSSMF_EINVAL, "child update index outside the parent front");
          m[t] = F.s + (int)(it - F.upd.begin());
        }
      }
      F.kidmap.push_back(std::move(m));
    }
  }
  int maxh = 0;
  for (auto& F : P.fr) maxh = std::max(maxh, F.height);
  P.levels.assign(nf ? maxh + 1 : 0, {});
  for (auto& F : P.fr) P.levels[F.height].push_back(F.id);
}

void front_local_csr(const Plan& P, const FrontPlan& f, bool transpose, LocalCSR& out) {
  // triplets (local row, local col, value index) of A_i
  auto local = [&](int j) -> int {
    if (j >= f.lo && j < f.hi) return j - f.lo;
    auto it = std::lower_bound(f.upd.begin(), f.upd.end(), j);
    if (it != f.upd.end() && *it == j) return f.s + (int)(it - f.upd.begin());
    return -1;
  };
  std::vector<std::vector<std::pair<int, int64_t>>> rows(f.n);
  for (int i = f.lo; i < f.hi; ++i) {
    int r = i - f.lo;
    for (int64_t e = P.prow[i]; e < P.prow[i + 1]; ++e) {
      int c = local(P.pcol[e]);
      if (c >= 0) {
        if (!transpose) rows[r].push_back({c, P.pvidx[e]});
        else rows[c].push_back({r, P.pvidx[e]});
      }
    }
    // column i of A below: entries (row in I_upd, col i)
    for (int64_t e = P.trow[i]; e < P.trow[i + 1]; ++e) {
      int rr = local(P.tcol[e]);
      if (rr >= f.s) {
        if (!transpose) rows[rr].push_back({r, P.tvidx[e]});
        else rows[r].push_back({rr, P.tvidx[e]});
      }
    }
  }
  out.rowptr.assign(f.n + 1, 0);
  out.col.clear();
  out.vidx.clear();
  for (int r = 0; r < f.n; ++r) {
    std::sort(rows[r].begin(), rows[r].end());
    for (auto& t : rows[r]) {
      out.col.push_back(t.first);
      out.vidx.push_back(t.second);
    }
    out.rowptr[r + 1] = (int)out.col.size();
  }
}

}  // namespace hssmf
