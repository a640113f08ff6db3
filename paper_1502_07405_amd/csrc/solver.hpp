// Host-side structures of a factorization: symbolic plan, per-front device
// storage, HSS node storage.
#pragma once
#include <chrono>
#include <memory>
#include <vector>

#include "kernels.hpp"
#include "vec.hpp"

namespace hssmf {

// ------------------------------------------------------------- plan -------
struct FrontPlan {
  int id = 0, lo = 0, hi = 0, s = 0, u = 0, n = 0, parent = -1, height = 0;
  bool hss = false;
  std::vector<int> kids;
  std::vector<int> upd;                 // sorted new indices of I_upd
  std::vector<std::vector<int>> kidmap; // per kid: kid-local update index -> local index here
};

struct Plan {
  int n = 0, nfront = 0;
  int64_t nnz = 0;
  std::vector<int> perm, iperm;
  // P A P^T in CSR (new indices); pvidx points into the caller's value array
  std::vector<int64_t> prow;
  std::vector<int> pcol;
  std::vector<int64_t> pvidx;
  // transpose structure of P A P^T
  std::vector<int64_t> trow;
  std::vector<int> tcol;
  std::vector<int64_t> tvidx;
  std::vector<FrontPlan> fr;
  std::vector<std::vector<int>> levels;  // by height, 0 = leaves
};

void build_plan(const hssmf_csr* A, const hssmf_ordering* ord, const hssmf_opts* o, Plan& P);

// front-local CSR of A_i: rows with local index < s keep every entry inside
// the front, rows >= s keep the entries in columns < s (Eq. frontal_1)
struct LocalCSR {
  std::vector<int> rowptr, col;
  std::vector<int64_t> vidx;
};
void front_local_csr(const Plan& P, const FrontPlan& f, bool transpose, LocalCSR& out);

// ----------------------------------------------------------- HSS nodes -----
struct HNode {
  int lo = 0, hi = 0, parent = -1, height = 0;
  int kid[2] = {-1, -1};
  bool leaf() const { return kid[0] < 0; }
  int m() const { return hi - lo; }
  // compression state
  bool done = false;
  int r = 0, c = 0, mr = 0, mc = 0;
  std::vector<int> permr, permc, Ir, Ic;  // host copies (local to the front)
  int *dpermr = nullptr, *dpermc = nullptr, *dIr = nullptr, *dIc = nullptr;
  int *drank = nullptr;                   // 2 ints: r, c
  double *D = nullptr, *B12 = nullptr, *B21 = nullptr;
  double *Er = nullptr, *Ec = nullptr;
  double *Sr = nullptr, *Sc = nullptr;            // node samples (before the ID)
  double *Srr = nullptr, *Scr = nullptr, *Rrr = nullptr, *Rcr = nullptr;  // reduced
  // ULV
  int nl = 0;
  double *Q = nullptr, *L = nullptr, *WQ = nullptr, *QV = nullptr;  // Q: Qtilde^T; D21|Dh = WQ, V1;Vh = QV
  double *Dbar = nullptr, *Vbar = nullptr;
  double *Ud = nullptr, *Vd = nullptr;    // dense interpolative generators
  double *Ubig = nullptr, *Vbig = nullptr;
  // non-leaf nodes of an update subtree kept in low-rank form: B12 Vbig_b^T
  // (r_a x m_b) and B21 Vbig_a^T (r_b x m_a), for entry extraction
  double *T12 = nullptr, *T21 = nullptr;
  // solve buffers (fixed addresses, so the solve launches are built once)
  double *bbar = nullptr, *ctop = nullptr, *cbot = nullptr, *w = nullptr, *wab = nullptr;
  double *xin = nullptr, *xbar = nullptr, *gt = nullptr, *gbar = nullptr, *lbar = nullptr, *hv = nullptr;
  double *tmp1 = nullptr, *tmpv = nullptr;
  int* diperm = nullptr;      // inverse of permr
};

struct HFront {
  int f = 0, n = 0, s = 0, u = 0;
  std::vector<HNode> nd;
  int root = -1, k = -1, q = -1, maxh = 0;
  // sampling
  int d = 0, dcap = 0, rounds = 0, swaps = 0;   // swaps: strong-RRQR interchanges
  double *R = nullptr, *Sr = nullptr, *Sc = nullptr;
  // power iteration: R^r (row side) and R^c (column side) of Alg. 1, n x
  // dcap like R; nullptr for plain sampling, where both are R
  double *Rr = nullptr, *Rc = nullptr;
  const double* rr() const { return Rr ? Rr : R; }
  const double* rc() const { return Rc ? Rc : R; }
  void* Rlp = nullptr;       // low-precision copy of R (mixed precision)
  int* orig = nullptr;       // original row ids of the front's indices
  bool finished = false, refresh = false;
  // front operator
  int *a_row = nullptr, *a_col = nullptr, *at_row = nullptr, *at_col = nullptr;
  int64_t *a_vidx = nullptr, *at_vidx = nullptr;
  int fop = -1;
  // ULV top node and low-rank Schur complement
  double* Dk = nullptr;
  int* ipivk = nullptr;
  int mk = 0;
  double *Vbark = nullptr, *ThT = nullptr, *Phi = nullptr;
  double* Upd = nullptr;     // dense update matrix (u x u)
  // the update matrix reaches the (HSS) parent in low-rank form: the
  // q-subtree generators with Theta^* and Phi, kept until the parent is done
  bool lowrank = false;
  struct HssKidDev* kdev = nullptr;   // device table for entry extraction
  // copies kept for inspection when opts.keep_stages is set: R, S^r, S^c at
  // the final d (n x kd each), Theta^T and Phi (mk x u each)
  double *kR = nullptr, *kSr = nullptr, *kSc = nullptr, *kTh = nullptr, *kPhi = nullptr;
  int kd = 0;
  void* UpdLP = nullptr;     // low-precision copy for sampling GEMMs
  double *X = nullptr, *t1 = nullptr, *t2 = nullptr;  // solve buffers
};

// one recorded launch of the solve phase
struct Op {
  int kind;      // OP_*
  const void* d; // device descriptor array
  int n;         // descriptors
  int64_t p0;    // kernel parameter (max extent / trsv kind)
  // triangular solves with one workgroup per block of 64 entries: their
  // launch-count, ticket and flag words (nullptr: one workgroup per system)
  int* ws = nullptr;
};
enum { OP_GEMV = 0, OP_COPY = 1, OP_TRSV = 2, OP_RHS = 3 };

// ---------------------------------------------------------- fronts ---------
struct FrontRT {
  // dense front storage (whole front kept: F11 = L\U, F12 = U12, F21 = L21,
  // F22 = update matrix until the parent consumed it)
  double* F = nullptr;
  int* ipiv = nullptr;
  // update matrix seen by the parent
  const double* U = nullptr;
  int ldu = 0;
  const void* Ulp = nullptr;  // low-precision copy (HSS parents in mixed mode)
  int* d_upd = nullptr;       // global new indices of I_upd
  int* d_kidmap[2] = {nullptr, nullptr};  // kid-local -> local (device)
  int* d_inv[2] = {nullptr, nullptr};     // local -> kid-local or -1 (device)
  double* w = nullptr;        // forward-sweep update vector (u)
  int hidx = -1;              // index into Handle::hf for HSS fronts
  int64_t asm_off = 0, asm_cnt = 0;  // range in the assembly map arrays
};

// Progress of the stepwise interpolative decompositions as the host sees it
// without synchronizing: the stop step of every problem sets that problem's
// flag in mapped, coherent pinned memory, and a ring of stream events (one
// recorded every kEvery pivot steps) bounds how far the host runs ahead of
// the device.
struct IdPoll {
  static constexpr int kEvery = 8;   // pivot steps per recorded event
  static constexpr int kRing = 2;    // events in the ring: the host leads by < kRing * kEvery + kEvery steps
  int* host = nullptr;               // flags as the host reads them
  int* dev = nullptr;                // the same flags as the device writes them
  size_t cap = 0;
  hipEvent_t ev[kRing] = {};
  bool armed[kRing] = {};
  void reserve(size_t n) {
    if (!ev[0])
      for (auto& e : ev) HIP_CHECK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    if (n <= cap) return;
    if (host) HIP_CHECK(hipHostFree(host));
    host = dev = nullptr;
    cap = 0;
    HIP_CHECK(hipHostMalloc((void**)&host, n * sizeof(int), hipHostMallocMapped | hipHostMallocCoherent));
    HIP_CHECK(hipHostGetDevicePointer((void**)&dev, host, 0));
    cap = n;
  }
  // after pivot step t has been enqueued: every kEvery steps, wait for the
  // event recorded kRing * kEvery steps ago, then record a new one
  void pace(int t, hipStream_t s) {
    if (t % kEvery != kEvery - 1) return;
    const int k = (t / kEvery) % kRing;
    if (armed[k]) HIP_CHECK(hipEventSynchronize(ev[k]));
    HIP_CHECK(hipEventRecord(ev[k], s));
    armed[k] = true;
  }
  void reset() {
    for (auto& a : armed) a = false;
  }
  ~IdPoll() {
    for (auto& e : ev)
      if (e) (void)hipEventDestroy(e);
    if (host) (void)hipHostFree(host);
  }
};

// GMRES progress in mapped, coherent pinned host memory: the device's
// Givens step stores each Arnoldi step's residual estimate and tag there,
// and the host waits for the tag without draining the stream
struct GmPoll {
  GmStatus* host = nullptr;
  GmStatus* dev = nullptr;
  int tag = 0;
  void init() {
    if (host) return;
    HIP_CHECK(hipHostMalloc((void**)&host, sizeof(GmStatus), hipHostMallocMapped | hipHostMallocCoherent));
    HIP_CHECK(hipHostGetDevicePointer((void**)&dev, host, 0));
    host->est = 0.0;
    host->tag = 0;
  }
  // the estimate of the step tagged t, once the device has stored it
  double wait(int t) {
    const auto t0 = std::chrono::steady_clock::now();
    for (unsigned spin = 0;; ++spin) {
      if (__atomic_load_n(&host->tag, __ATOMIC_ACQUIRE) == t) return *(volatile double*)&host->est;
      if ((spin & 1023) == 1023 && std::chrono::steady_clock::now() - t0 > std::chrono::seconds(120))
        throw Error(HSSMF_EDEVICE, "GMRES: no Arnoldi step result from the device");
    }
  }
  ~GmPoll() {
    if (host) (void)hipHostFree(host);
  }
};

struct Handle {
  Plan P;
  hssmf_opts o{};
  hipStream_t st = nullptr;
  Arena arena;       // plan data that survives refactorization
  Arena narena;      // numeric factors, reset by every refactorization
  Arena larena;      // compression state of one elimination-tree level
  Arena sarena;      // temporaries of one batched pass (stream ordered reuse)
  Arena* cur = &arena;
  Stager stager;
  IdPoll idpoll;
  GmPoll gmpoll;
  // set by a device wait that gave up (mapped, host-coherent); checked once
  // an entry point has synchronized its stream
  int* werr_h = nullptr;
  int* werr_d = nullptr;
  // pinned host words for the results the host reads back after a pass
  // (device-to-host copies into it stay asynchronous, so a pass's several
  // read-backs cost one stream synchronization)
  int* pin = nullptr;
  size_t pin_cap = 0;
  int* pinned_ints(size_t n) {
    if (n > pin_cap) {
      if (pin) HIP_CHECK(hipHostFree(pin));
      pin = nullptr;
      pin_cap = std::max<size_t>(n, 2 * pin_cap);
      HIP_CHECK(hipHostMalloc((void**)&pin, pin_cap * sizeof(int), hipHostMallocDefault));
    }
    return pin;
  }
  GmDev gm{};                  // GMRES state on the device
  std::vector<Op> sops[2][2];  // [trans][0 = forward, 1 = backward]
  // status of the last numeric factorization: HSSMF_OK when the factors and
  // the recorded solve operations are valid, else the error it ended with
  // (the solve entry points return it and launch nothing)
  int factor_status = HSSMF_EINVAL;
  double* yws = nullptr;       // n, the right-hand side in the new ordering
  int* d_iperm = nullptr;
  int *d_row = nullptr, *d_col = nullptr;  // CSR entry coordinates (adjoint)
  int64_t *d_trowptr = nullptr, *d_tvidx = nullptr;  // A^T in CSR (original order)
  int* d_tcolind = nullptr;
  double* d_scal = nullptr;    // device scalars of the outer solvers
  double* d_part = nullptr;    // dot-product partial sums
  int device = 0;
  double* d_val = nullptr;    // caller's CSR values (original order)
  int64_t* d_rowptr = nullptr;
  int* d_colind = nullptr;
  int* d_perm = nullptr;
  int64_t* d_asm_dst = nullptr;  // assembly: front element offset (relative to the level buffer)
  int64_t* d_asm_src = nullptr;  // assembly: value index
  std::vector<double*> level_buf;
  std::vector<FrontRT> fr;
  std::vector<HFront> hf;
  int* d_info = nullptr;
  int failed_front = -1;
  double* vec_ws = nullptr;   // solve workspace (n doubles x several)
  // independent systems factored together (hssmf_factor_batch): unknowns
  // [sys_off[s], sys_off[s+1]) belong to system s; one system otherwise
  std::vector<int64_t> sys_off;
  // a complex system factored through its real-equivalent form
  // (hssmf_factor_z): the complex CSR's row pointers, base 0
  bool zexp = false;
  std::vector<int64_t> zrow;
  int64_t* d_zrow = nullptr;   // the same on the device (arena)
  int64_t* d_sys_off = nullptr;
  double* d_seg = nullptr;     // per-system sums of squares
  // preconditioner sweeps captured as HIP graphs ([trans]), rebuilt after
  // every numeric factorization; captured on a private stream
  hipGraphExec_t gexec[2] = {nullptr, nullptr};
  hipStream_t gst = nullptr;
  // streams beside st for launches of one pass that may run side by side
  // (default priority, created on first use), with the events that fork
  // them from st and join them back
  static constexpr int kAux = 3;
  hipStream_t aux[kAux] = {};
  hipEvent_t ev_fork = nullptr, ev_join[kAux] = {};
  void make_aux() {
    if (ev_fork) return;
    for (int i = 0; i < kAux; ++i) {
      HIP_CHECK(hipStreamCreateWithFlags(&aux[i], hipStreamNonBlocking));
      HIP_CHECK(hipEventCreateWithFlags(&ev_join[i], hipEventDisableTiming));
    }
    HIP_CHECK(hipEventCreateWithFlags(&ev_fork, hipEventDisableTiming));
  }
  void drop_graphs() {
    for (auto& g : gexec)
      if (g) { (void)hipGraphExecDestroy(g); g = nullptr; }
  }
  ~Handle() {
    drop_graphs();
    if (gst) (void)hipStreamDestroy(gst);
    for (int i = 0; i < kAux; ++i) {
      if (aux[i]) (void)hipStreamDestroy(aux[i]);
      if (ev_join[i]) (void)hipEventDestroy(ev_join[i]);
    }
    if (ev_fork) (void)hipEventDestroy(ev_fork);
    if (werr_h) (void)hipHostFree(werr_h);
    if (pin) (void)hipHostFree(pin);
  }
  hssmf_stats stats{};
  GemmType gt() const;
  // products of the low-rank Schur update and of its dense expansion:
  // FP64 operands rounded to FP32 on the matrix cores in the low-precision
  // modes, FP64 otherwise
  GemmType gs() const { return o.gemm_prec == HSSMF_PREC_FP64 ? GEMM_F64 : GEMM_D_F32; }
};

void numeric_factor(Handle& h);
// y = M^{-1} x or M^{-T} x; graph = false keeps the sweeps eager even when
// use_graph is set (no capture, nothing allocated)
void apply_inverse(Handle& h, int trans, const double* x, double* y, bool graph = true);
void spmv(Handle& h, int trans, const double* x, double* y, double alpha, double beta);
// the outer solver of the options on one right-hand side (device b, x):
// work vectors from the handle's arena (ws null) or carved from ws (wscap
// doubles; the sweeps then run eagerly); returns HSSMF_OK / HSSMF_ENOCONV,
// throws Error otherwise
int outer_solve(Handle& h, int trans, const double* b, double* x, hssmf_info* info, double* ws = nullptr,
                size_t wscap = 0);
// doubles of workspace outer_solve takes for n unknowns under options o
size_t outer_workspace(const hssmf_opts& o, int64_t n);
double dnrm2(Handle& h, const double* x, int n);

// device helpers shared by factor and solve
void blocked_lu(Handle& h, const std::vector<LUFront>& fronts);
void tri_solve_many(Handle& h, const double* T, int ldt, int n, double* X, int ldx, int ncols, bool lower,
                    bool unit, bool trans);

struct TriProb {
  const double* T;
  int ldt, n;
  double* X;
  int ldx, ncols;
};
void tri_solve_upper_batched(Handle& h, const std::vector<TriProb>& ps);

void build_solve_ops(Handle& h);
void run_ops(Handle& h, const std::vector<Op>& ops);

template <class T>
T* upload(Handle& h, const std::vector<T>& v) {
  T* d = h.cur->get<T>(v.size());
  if (!v.empty()) h.stager.put_to(d, v.data(), v.size() * sizeof(T), h.st);
  return d;
}

}  // namespace hssmf
