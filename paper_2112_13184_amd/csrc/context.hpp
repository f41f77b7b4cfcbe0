// CTMRG context: resident environment, workspaces and the sweep driver.
#pragma once

#include <algorithm>
#include <array>
#include <atomic>
#include <complex>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/ctm.h"
#include "common.hpp"
#include "gemm.hpp"
#include "linalg.hpp"
#include "smallla.hpp"

namespace ctm {

// Bump allocator for the transient tensors of the expectation-value
// contractions: a list of device chunks, reused after reset().  The first
// chunk has first_elems elements (the expected peak); release() rolls back to
// a mark (work already enqueued on the context's stream still reads the
// released memory before any later kernel can overwrite it).
struct Arena {
  std::vector<DevBuf*> chunks;
  size_t cur = 0, used = 0;   // current chunk, elements used in it
  size_t first_elems = 0;
  // While ext is set, alloc() bumps through this fixed device buffer instead
  // of the chunks (it never allocates then, and throws CTM_ETOOBIG when the
  // buffer is full); `used` is the offset into it.
  double* ext = nullptr;
  size_t ext_elems = 0;
  double* alloc(size_t elems);
  void reset() { cur = 0; used = 0; }
  std::array<size_t, 2> mark() const { return {cur, used}; }
  void release(const std::array<size_t, 2>& m) { cur = m[0]; used = m[1]; }
  size_t bytes() const {
    size_t b = 0;
    for (auto* c : chunks) b += c->bytes;
    return b;
  }
  ~Arena() { for (auto* b : chunks) delete b; }
};

// Device tensor view (row-major).
struct DT {
  double* p = nullptr;
  std::vector<long> dims;
  long size() const {
    long s = 1;
    for (long d : dims) s *= d;
    return s;
  }
};

// Per-phase launch timing with HIP events on the context stream.
struct PhaseTimer {
  enum { EDGE = 0, SKETCH = 1, ABSORB = 2, LINALG = 3, OTHER = 4, N = 5 };
  // phases timed (bit per phase); each pair of events leaves a dispatch gap
  // of about 10 us on the stream, so a run can time its dominant phase only
  unsigned mask = 0;
  // an open group (one pair of events around several launches of a phase):
  // the timed() calls inside it add their launches and flops to it
  bool grouped = false;
  int group_phase = 0;
  int64_t group_launches = 0;
  double group_flops = 0.0;
  std::vector<hipEvent_t> pool;
  size_t next = 0;
  struct Rec { int phase; hipEvent_t a, b; double flops; int64_t launches; };
  std::vector<Rec> recs;
  int64_t launches[N] = {};
  double ms[N] = {}, flops[N] = {};
  hipEvent_t get() {
    if (next == pool.size()) {
      hipEvent_t e;
      CTM_HIP(hipEventCreate(&e));
      pool.push_back(e);
    }
    return pool[next++];
  }
  void clear() {
    recs.clear();
    next = 0;
    for (int i = 0; i < N; ++i) { launches[i] = 0; ms[i] = 0; flops[i] = 0; }
  }
  void resolve() {
    for (auto& r : recs) {
      float t = 0.f;
      CTM_HIP(hipEventSynchronize(r.b));
      CTM_HIP(hipEventElapsedTime(&t, r.a, r.b));
      launches[r.phase] += r.launches;
      ms[r.phase] += t;
      flops[r.phase] += r.flops;
    }
    recs.clear();
    next = 0;
  }
  ~PhaseTimer() { for (auto e : pool) (void)hipEventDestroy(e); }
};

struct Context {
  ctm_config cfg{};
  PhaseTimer timer;
  int Lx = 0, Ly = 0, N = 0;  // unit cell and its number of sites
  // Replicas: R independent solves of the same shape in one context.  Replica
  // r owns the sites r*N .. r*N+N-1 of every per-site buffer; the cuts of a
  // column of all replicas are batched into the same launches.
  int R = 1;
  int NS() const { return R * N; }
  std::vector<uint64_t> seeds;   // sketch seed per replica
  std::vector<long long> rmoves; // moves done by each replica (keys its sketch streams)
  std::vector<char> frozen;      // replica no longer updated (converged, capped, cancelled, failed)
  // NaN / Inf or a cut without singular values in a replica's last move.  A
  // context with isolate set records it here (and the caller freezes the
  // replica); otherwise the move throws CTM_ENUMERIC.
  std::vector<char> failed;
  bool isolate = false;
  int device = 0;            // HIP device the context lives on
  int D = 0, d = 0, DK = 0, DB = 0, Db = 0, chi = 0, n = 0, layers = 2;
  int kk = 0;               // sketch width
  double cutoff = 1e-12;
  hipStream_t st = nullptr;
  bool own_stream = false;
  Linalg* la = nullptr;
  SmallLA sla;
  std::string err;
  long long moves = 0;

  // site tensors, four rotations each: [rot][site][...]
  DevBuf Aket, Abra;
  long szk = 0, szb = 0;    // elements per site tensor (ket / bra)
  // environment: [site][k][...]
  DevBuf envC, envTa, envTb;
  // leg dims (host): cdim[site][k][0..1] = (next, prev); tdim[site][k][0..1] = (prev, next)
  std::vector<std::array<std::array<int, 2>, 4>> cdim, tdim;

  // absorption offset tables
  DevBuf ketA_r, ketA_c, ketC_r, ketC_c, braB_r, braB_c, braCn_r, braCn_c, braCt_r, braCt_c;

  // workspaces
  // the four corner roles [role][slot][n][n], one allocation (so that batched
  // launches address any corner by an offset from one base)
  DevBuf Gall;
  struct View {
    void* p = nullptr;
    template <typename T> T* as() const { return static_cast<T*>(p); }
  } G[4];
  DevBuf X1, X2, Ybuf;
  DevBuf pan[8];             // n x kk panels
  DevBuf small[6];           // kk x kk
  DevBuf Svals, wvec, keff, badflag, redscratch, delta;
  DevBuf Pt, PT, P3;         // [Ly][n][chi]
  DevBuf newC1, newT4, newC4;
  DevBuf spec, specprev, cornerscratch;
  DevBuf specws;             // convergence state of the corner-spectra Jacobi (64 problems)
  DevBuf gws;                // GEMM split-K workspace
  // Per-problem pointer tables of batched launches (corners and column
  // updates of several cuts, whose tensors are not evenly spaced): a ring of
  // 8-byte words on the device, filled by stream-ordered copies from a pinned
  // host ring.  The host ring is reused only after the stream has drained.
  DevBuf ptab;
  PinnedBuf ptab_host;
  // pinned staging for the small device-to-host reads of the host logic
  // (failure flags, deltas, observables): stream-ordered DMA, no pageable
  // staging inside the runtime
  PinnedBuf hpin;
  size_t ptab_words = 0, ptab_used = 0;
  int bchunk = 1;            // problems per batched corner / update launch (n x n scratch each)
  size_t gws_elems = 0;
  DevBuf amax;               // split-FP16 operand scaling (2 words)
  DevBuf camax;              // split FP16: largest |entry| of each corner role over a column's cuts
  // BF16 / split FP16: the corners of a column's cuts and the sketch panels
  // stored once in the reduced type (gemm_pre operands); lp_ld = their row pitch
  DevBuf Glp, panlp, panscale;
  DevBuf x2lp, x2rs;         // BF16 / split FP16 edge-corner product operands and their row scales
  long lp_ld = 0;
  int lp_npl = 0;
  GemmType ctype = GemmType::F64;   // arithmetic of the contraction GEMMs
  Arena arena;
  std::vector<int> nact_cut; // per slot of the current column: bond dim after the move
  std::vector<int> cut_slot; // (r * Lyv + y) -> slot of that cut in this column (-1: frozen)
  int64_t cuts[3] = {0, 0, 0}; // cuts by path: identity, batched randomized SVD, fallback
  bool last_cut_svd = false; // the last cut_projectors() call went through the SVD

  // helpers
  double* C(int s, int k) const { return envC.as<double>() + ((long)s * 4 + k) * chi * chi; }
  double* Ta(int s, int k) const { return envTa.as<double>() + ((long)s * 4 + k) * chi * chi * Db; }
  double* Tb(int s, int k) const { return envTb.as<double>() + ((long)s * 4 + k) * chi * chi * Db; }
  const double* Ak(int rot, int s) const { return Aket.as<double>() + ((long)rot * NS() + s) * szk; }
  const double* Ab(int rot, int s) const { return Abra.as<double>() + ((long)rot * NS() + s) * szb; }
  GemmWorkspace ws() const { return GemmWorkspace{gws.as<double>(), gws_elems, amax.as<unsigned>()}; }
};

// dst[0..n) = src[0..n) (device) through the context's pinned buffer, after
// the work enqueued on the context's stream; synchronises the stream.
template <typename T>
void d2h(Context& c, T* dst, const T* src, size_t n) {
  const size_t chunk = c.hpin.bytes / sizeof(T);
  for (size_t o = 0; o < n; o += chunk) {
    const size_t m = std::min(chunk, n - o);
    CTM_HIP(hipMemcpyAsync(c.hpin.p, src + o, m * sizeof(T), hipMemcpyDeviceToHost, c.st));
    CTM_HIP(hipStreamSynchronize(c.st));
    std::memcpy(dst + o, c.hpin.p, m * sizeof(T));
  }
}

// Run f (which enqueues work on c.st) inside a timed region of `phase`.
template <typename F>
inline void timed(Context& c, int phase, double flops, F&& f) {
  PhaseTimer& t = c.timer;
  if (!(t.mask >> phase & 1u)) {
    f();
    return;
  }
  if (t.grouped) {
    f();
    if (phase == t.group_phase) {
      t.group_launches += 1;
      t.group_flops += flops;
    }
    return;
  }
  hipEvent_t a = t.get(), b = t.get();
  CTM_HIP(hipEventRecord(a, c.st));
  f();
  CTM_HIP(hipEventRecord(b, c.st));
  t.recs.push_back({phase, a, b, flops, 1});
}

// One pair of events around f, whose timed() launches of `phase` are counted
// in it (launches of other phases inside f are not timed).
template <typename F>
inline void timed_group(Context& c, int phase, F&& f) {
  PhaseTimer& t = c.timer;
  if (!(t.mask >> phase & 1u) || t.grouped) {
    f();
    return;
  }
  hipEvent_t a = t.get(), b = t.get();
  CTM_HIP(hipEventRecord(a, c.st));
  t.grouped = true;
  t.group_phase = phase;
  t.group_launches = 0;
  t.group_flops = 0.0;
  f();
  t.grouped = false;
  CTM_HIP(hipEventRecord(b, c.st));
  t.recs.push_back({phase, a, b, t.group_flops, t.group_launches});
}

// tensors: `replicas` sets of Lx*Ly site tensors, one after the other;
// seeds: one sketch seed per replica (nullptr: cfg.seed for all).
void context_init(Context& c, const ctm_config& cfg, const double* tensors, int on_device,
                  const double* boundary, int replicas = 1, const uint64_t* seeds = nullptr);
size_t context_footprint(const ctm_config& cfg);
// Footprint of a context holding `replicas` solves of this configuration.
size_t context_footprint_group(const ctm_config& cfg, int replicas);
void do_move(Context& c, int rot);
// Up to max_sweeps sweeps, stopping when delta < tol or when *cancel (checked
// before every sweep) becomes true.
void do_sweeps(Context& c, int max_sweeps, double tol, int* done, double* delta, int* converged,
               const std::atomic<bool>* cancel = nullptr);
// The context inside a handle of the C ABI.
Context& context_of(ctm_ctx* ctx);
// A handle holding `replicas` solves of one configuration (tensors: replicas
// sets of Lx*Ly host site tensors; seeds: one per replica).  nullptr with
// *st set on failure; released with ctm_free.
ctm_ctx* create_group(const ctm_config& cfg, const double* tensors, int replicas, const uint64_t* seeds,
                      ctm_status* st);
void cut_projectors(Context& c, int rot, int r, int x, int y, int slot);
void cut_projectors_fast(Context& c, int rot, int x, int y);
// Sweeps of every replica until each converges (delta < tol[r]), reaches
// max_sweeps[r] or is cancelled (cancel[r], checked before every sweep); a
// finished replica is frozen.  done / delta / converged: one entry per replica.
void do_sweeps_group(Context& c, const int* max_sweeps, const double* tol, int* done, double* delta,
                     int* converged, const std::atomic<bool>* const* cancel);
// The steps of do_sweeps_group, for a caller that drives the replicas itself
// (the serving queue): group_start takes the reference corner spectra of
// every replica; group_sweep runs one sweep of the live replicas and returns
// each replica's delta in host_delta (R values; entries of frozen replicas
// are not meaningful).  replica_reset starts a new solve in slot r (site
// tensors, trivial environment, reference spectra, move count, seed).
void group_start(Context& c);
void group_sweep(Context& c, double* host_delta);
void replica_reset(Context& c, int r, const double* tensors_host, uint64_t seed);
void enlarged_corner(Context& c, int s, int j, double* out, unsigned* amax = nullptr);
// Reduced density matrices, normalised to trace 1, in the device buffer
// rho_dev (d*d or d^4 doubles); copied to rho_host when it is not null.
void rho_1site(Context& c, int site, double* rho_dev, double* rho_host);
void rho_2site(Context& c, int site, int dir, double* rho_dev, double* rho_host);
// sum_{i,o} rho[i][o] op[o][i] for a dim x dim operator (host), on the device.
double expect_op(Context& c, const double* rho_dev, const double* op_host, int dim);
// <O> on one site and <h> on the bond (site, site + x) (dir 0) or (site, site + y)
// (dir 1), contracting the operator into closed networks instead of forming
// the reduced density matrix (op layout [out][in], as for rho).
double expect_1site(Context& c, int site, const double* op_host, int replica = 0);
double expect_2site(Context& c, int site, int dir, const double* op_host, int replica = 0);
// Elements of the largest transient the expectation values above (and the
// classical impurity / ln kappa) allocate.
size_t observe_arena_elems(long chi, long DK, long DB, long d);
double impurity(Context& c, int site, const double* b_host);
// C(r) = <A(site) B(site + r e)> for r = 0..rmax (out, host), e = +x (dir 0)
// or +y (dir 1); operators [out][in], host.
void correlation(Context& c, int site, int dir, const double* opA, const double* opB, int rmax, double* out);
// The nev eigenvalues of largest modulus of the transfer matrix of one
// period along +x (dir 0, in row `line`) or +y (dir 1, in column `line`), by
// explicitly restarted Arnoldi (Krylov dimension `krylov`, Ritz residual
// tolerance tol relative to |lambda_0|); sorted by modulus, descending.
// Returns the number of restarts.
int transfer_spectrum(Context& c, int dir, int line, int nev, int krylov, double tol, std::complex<double>* lam);
double log_kappa(Context& c);
// numpy.tensordot / transpose of device tensors, results in c.arena (FP64).
DT tensordot(Context& c, const DT& A, const std::vector<int>& axA, const DT& B, const std::vector<int>& axB);
DT tensor_transpose(Context& c, const DT& A, const std::vector<int>& perm);
// Full update: N[(rho_i, rho_j)][(rho_i', rho_j')] of the bond (site, site + x)
// (dir 0) or (site, site + y) (dir 1), the bond-density-matrix patch of the
// environment with the tensors Ei, Ej ([l][u][r][d][rho], rho of dimension r,
// device, physical frame) in place of the two sites; trace 1, in c.arena.
DT bond_environment(Context& c, int site, int dir, const double* Ei, const double* Ej, int r);
// exp(-tau_b H) of batch x N x 2 bond Hamiltonians (d2 x d2, device) on st.
void trotter_gates(hipStream_t st, const double* H, const double* tau, double* gates, int N, int d2, int batch);
// One full-update Trotter step (bond Hamiltonians H [N][2][d^2][d^2], host).
void full_update_step(Context& c, const double* H, double tau, int als_iters, int env_sweeps);
// Site tensors of every site (rotation 0) to host memory.
void get_site_tensors(Context& c, double* out);
void check_bad(Context& c, const char* where);

}  // namespace ctm
