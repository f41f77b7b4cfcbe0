// Directional moves and sweeps of the CTMRG (Sec. 2.2 of arXiv:2112.13184).
//
// Layout in HBM (FP64, zero padded to chi on every chi leg):
//   envC [site][k][chi][chi]          C_k[next][prev]
//   envTa[site][k][chi][chi][Db]      T_k[prev][next][pair]   (edge as "next" of a corner)
//   envTb[site][k][chi][Db][chi]      T_k[prev][pair][next]   (edge as "prev" of a corner)
//   Aket / Abra [rot][site][...]      site tensor seen from corner rot (rotated rot
//                                     quarter turns counter-clockwise)
// Both edge layouts are kept so that every edge contraction is a plain GEMM.
//
// A move in direction `rot` is a left move on the lattice rotated rot quarter
// turns: view corner m is physical corner (m + rot) % 4, the same for edges.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "absorb.hpp"
#include "context.hpp"
#include "kernels.hpp"
#include "smallla.hpp"

namespace ctm {

namespace {

inline int mod(int a, int b) { return ((a % b) + b) % b; }

// CTM_DEBUG=1 in the environment prints the projector path taken per column.
const bool g_debug = getenv("CTM_DEBUG") != nullptr;

// Physical site of view position (xv, yv) in the frame rotated rot quarter turns.
int view_site(const Context& c, int rot, int xv, int yv) {
  int x = xv, y = yv;
  for (int i = 0; i < rot; ++i) { int t = x; x = y; y = -t; }
  return mod(x, c.Lx) + c.Lx * mod(y, c.Ly);
}

void view_dims(const Context& c, int rot, int& Lxv, int& Lyv) {
  Lxv = (rot % 2 == 0) ? c.Lx : c.Ly;
  Lyv = (rot % 2 == 0) ? c.Ly : c.Lx;
}

uint64_t stream_id(long long move, int x, int y) {
  return ((uint64_t)(move & 0xFFFFFFFFll) << 32) | ((uint64_t)(x & 0xFFFF) << 16) | (uint64_t)(y & 0xFFFF);
}

// Rotate a site tensor t[l][u][r][d][p] (dims Dd) one quarter turn
// counter-clockwise: out[a][b][c][e][p] = in[e][a][b][c][p].
// Batched corner and column-update launches give every problem its own n x n
// and chi x n scratch; at most this much n x n scratch in all (one problem
// per launch once n x n alone exceeds half of it: large n gains nothing from
// batching, its launches are long).
constexpr size_t kBatchScratchBytes = (size_t)256 << 20;
constexpr size_t kTableWords = (size_t)1 << 18;   // pointer-table ring: 2 MiB

long batch_chunk(long nn, long slots) {
  const long by_mem = (long)(kBatchScratchBytes / ((size_t)nn * sizeof(double)));
  return std::max<long>(1, std::min<long>(by_mem < 2 ? 1 : by_mem, 4 * slots));
}

void rotate_host(const std::vector<double>& in, std::vector<double>& out, int Dd, int d) {
  out.resize(in.size());
  for (int a = 0; a < Dd; ++a)
    for (int b = 0; b < Dd; ++b)
      for (int cc = 0; cc < Dd; ++cc)
        for (int e = 0; e < Dd; ++e)
          for (int p = 0; p < d; ++p)
            out[(((a * Dd + b) * Dd + cc) * Dd + e) * d + p] = in[(((e * Dd + a) * Dd + b) * Dd + cc) * d + p];
}

void upload_tables(DevBuf& buf, const std::vector<int>& v) {
  buf.alloc(v.size() * sizeof(int));
  CTM_HIP(hipMemcpy(buf.p, v.data(), v.size() * sizeof(int), hipMemcpyHostToDevice));
}

// Offset tables of the two absorption GEMMs (see absorb()).
void build_tables(Context& c) {
  const int chi = c.chi, DK = c.DK, DB = c.DB, Db = c.Db, d = c.d;
  const long n = c.n;
  std::vector<int> v;
  // ket: rows m = (cp, l', cn, u'), k = (l, u), cols = (r, dd, p)
  v.resize((size_t)chi * DB * chi * DB);
  for (int cp = 0; cp < chi; ++cp)
    for (int lb = 0; lb < DB; ++lb)
      for (int cn = 0; cn < chi; ++cn)
        for (int ub = 0; ub < DB; ++ub)
          v[(((size_t)cp * DB + lb) * chi + cn) * DB + ub] = (int)((cp * (long)Db + lb) * n + cn * (long)Db + ub);
  upload_tables(c.ketA_r, v);
  v.resize((size_t)DK * DK);
  for (int l = 0; l < DK; ++l)
    for (int u = 0; u < DK; ++u) v[l * DK + u] = (int)(l * (long)DB * n + u * DB);
  upload_tables(c.ketA_c, v);
  const long ldy = (long)DB * DB * d;
  v.resize((size_t)chi * DB * chi * DB);
  for (int cp = 0; cp < chi; ++cp)
    for (int lb = 0; lb < DB; ++lb)
      for (int cn = 0; cn < chi; ++cn)
        for (int ub = 0; ub < DB; ++ub)
          v[(((size_t)cp * DB + lb) * chi + cn) * DB + ub] =
              (int)((cp * (long)chi + cn) * DK * DK * ldy + (lb * DB + ub) * d);
  upload_tables(c.ketC_r, v);
  v.resize((size_t)DK * DK * d);
  for (int r = 0; r < DK; ++r)
    for (int dd = 0; dd < DK; ++dd)
      for (int p = 0; p < d; ++p) v[(r * DK + dd) * d + p] = (int)((r * DK + dd) * ldy + p);
  upload_tables(c.ketC_c, v);
  // bra: rows m = (cp, cn, r, dd) (plain in Y), k = (l', u', p), cols = (r', d')
  v.resize((size_t)DB * DB * d);
  for (int lb = 0; lb < DB; ++lb)
    for (int ub = 0; ub < DB; ++ub)
      for (int p = 0; p < d; ++p) v[(lb * DB + ub) * d + p] = (int)((lb * DB + ub) * (long)DB * DB * d + p);
  upload_tables(c.braB_r, v);
  v.resize((size_t)DB * DB);
  for (int rb = 0; rb < DB; ++rb)
    for (int db = 0; db < DB; ++db) v[rb * DB + db] = (rb * DB + db) * d;
  upload_tables(c.braB_c, v);
  std::vector<int> vn((size_t)chi * chi * DK * DK), vt(vn.size());
  for (int cp = 0; cp < chi; ++cp)
    for (int cn = 0; cn < chi; ++cn)
      for (int r = 0; r < DK; ++r)
        for (int dd = 0; dd < DK; ++dd) {
          size_t m = (((size_t)cp * chi + cn) * DK + r) * DK + dd;
          vn[m] = (int)((cn * (long)Db + r * DB) * n + cp * (long)Db + dd * DB);
          vt[m] = (int)((cp * (long)Db + dd * DB) * n + cn * (long)Db + r * DB);
        }
  upload_tables(c.braCn_r, vn);
  upload_tables(c.braCt_r, vt);
  vn.assign((size_t)DB * DB, 0);
  vt.assign((size_t)DB * DB, 0);
  for (int rb = 0; rb < DB; ++rb)
    for (int db = 0; db < DB; ++db) {
      vn[rb * DB + db] = (int)(rb * n + db);
      vt[rb * DB + db] = (int)(db * n + rb);
    }
  upload_tables(c.braCn_c, vn);
  upload_tables(c.braCt_c, vt);
}

// BF16 and split FP16 runs of the batched randomized-SVD path (k <= the
// small-factorisation limit) keep the corners of a column's cuts and the
// sketch panels in the reduced type and multiply them with gemm_pre.
static bool uses_pre(const ctm_config& cfg, long kk) {
  return (cfg.prec == CTM_BF16 || cfg.prec == CTM_F16_SPLIT) && cfg.rsvd_oversample >= 0 &&
         cfg.projector_path == CTM_PATH_AUTO && kk <= kSmallLAMaxK;
}

struct Sizes {
  long n, nn, kk, chi, Db, y;
  size_t total_bytes;
};

Sizes sizes_of(const ctm_config& cfg, int R = 1) {
  Sizes s{};
  const long DK = cfg.D, DB = (cfg.layers == 2) ? cfg.D : 1;
  const long d = (cfg.layers == 2) ? cfg.d : 1;
  s.Db = DK * DB;
  s.chi = cfg.chi;
  s.n = s.chi * s.Db;
  s.nn = s.n * s.n;
  const int p = cfg.rsvd_oversample;
  s.kk = (p < 0) ? s.n : std::min<long>(s.chi + p, s.n);
  s.y = s.nn * d;
  const long N = (long)cfg.Lx * cfg.Ly * R, Lmax = (long)std::max(cfg.Lx, cfg.Ly) * R;   // sites, slots
  const long chi = s.chi, n = s.n, kk = s.kk, cc = chi * chi;
  // doubles, in the order context_init allocates them
  size_t e = 0;
  e += 4 * N * (DK * DK * DK * DK * d + DB * DB * DB * DB * d);   // site tensors, 4 rotations
  e += 4 * N * (cc + 2 * cc * s.Db);                               // C, T, transposed T
  const long bch = batch_chunk(s.nn, Lmax);                         // problems per batched launch
  e += 4 * s.nn * Lmax + bch * (chi * n + s.nn) + s.y;              // corners, X1, X2, Y
  e += 8 * n * kk * Lmax + 6 * kk * kk * Lmax;                      // panels, small matrices
  e += std::max(kk, n) * Lmax + chi * Lmax;                         // singular values, weights
  if (kk <= kSmallLAMaxK && p >= 0)                                 // Cholesky QR / Jacobi
    e += 6 * kk * kk * Lmax + kk * Lmax + n * kk * Lmax + 64 + 128;
  e += 3 * Lmax * n * chi + 2 * Lmax * cc + Lmax * cc * s.Db;       // projectors, new C / T
  e += 2 * 4 * N * chi + 4 * N * cc + 128;                          // spectra, corner scratch, its Jacobi state
  e += 8 * n * std::max(kk, chi) * R;                               // split-K partials
  e += 4096 + std::max<long>(2048, 1025 * Lmax) + 64;              // rho, reductions, flags
  e += kTableWords;                                                 // pointer tables
  e += observe_arena_elems(chi, DK, DB, d);                         // expectation values
  size_t b = 8 * e;
  if ((cfg.prec == CTM_BF16 || cfg.prec == CTM_F16_SPLIT) && chi <= 320) {   // edge-corner operands
    const size_t npl = (cfg.prec == CTM_F16_SPLIT) ? 2 : 1;
    b += 2 * npl * 2 * bch * n * pre_ld(chi) + 4 * 2 * bch * n;
  }
  if (uses_pre(cfg, kk)) {                                          // reduced-type corners and panels
    const size_t npl = (cfg.prec == CTM_F16_SPLIT) ? 2 : 1, ld = pre_ld(n);
    b += 2 * npl * (4 * Lmax * 2 * n * ld + Lmax * kk * ld) + 4 * Lmax * kk;
  }
  b += 4 * (size_t)(2 * cc * DB * DB + 2 * cc * DK * DK + 4 * DK * DK * d + 4 * DB * DB * d);  // tables
  b += 8 * (size_t)(4096 + 4096 * 64) + 4 * 4096;                   // Householder fallback buffers
  // per-context runtime overhead measured on MI355X (rocBLAS handle and its
  // workspace, stream, allocation granularity of ~70 buffers): 170-190 MiB
  b += (size_t)256 << 20;
  s.total_bytes = b;
  return s;
}

}  // namespace

double* Arena::alloc(size_t elems) {
  elems = ((elems + 31) / 32) * 32;
  if (ext) {
    CTM_CHECK(used + elems <= ext_elems, -5, "contraction needs more than the fixed scratch array");
    double* p = ext + used;
    used += elems;
    return p;
  }
  while (cur < chunks.size() && used + elems > chunks[cur]->bytes / sizeof(double)) {
    ++cur;
    used = 0;
  }
  if (cur == chunks.size()) {
    DevBuf* b = new DevBuf();
    try {
      b->alloc(std::max(elems, chunks.empty() ? first_elems : ((size_t)1 << 20)) * sizeof(double));
    } catch (...) {
      delete b;
      throw;
    }
    chunks.push_back(b);
    used = 0;
  }
  double* p = chunks[cur]->as<double>() + used;
  used += elems;
  return p;
}

size_t context_footprint(const ctm_config& cfg) { return sizes_of(cfg).total_bytes; }
size_t context_footprint_group(const ctm_config& cfg, int replicas) { return sizes_of(cfg, replicas).total_bytes; }

// Reads the per-replica NaN / Inf / zero flags of the kernels since the last
// check.  A flagged replica is recorded in c.failed; without isolation the
// call throws CTM_ENUMERIC instead.
void check_bad(Context& c, const char* where) {
  std::vector<int> bad(c.R, 0);
  d2h(c, bad.data(), c.badflag.as<int>(), c.R);
  bool any = false;
  for (int r = 0; r < c.R; ++r) {
    if (bad[r]) c.failed[r] = 1;
    any |= bad[r] != 0;
  }
  if (any) {
    CTM_HIP(hipMemsetAsync(c.badflag.p, 0, sizeof(int) * c.R, c.st));
    CTM_HIP(hipStreamSynchronize(c.st));
  }
  if (!c.isolate)
    for (int r = 0; r < c.R; ++r)
      if (c.failed[r]) {
        c.failed[r] = 0;
        throw Error(-4, std::string(where) + ": NaN/Inf or zero environment / cut");
      }
}

void context_init(Context& c, const ctm_config& cfg, const double* tensors, int on_device,
                  const double* boundary, int replicas, const uint64_t* seeds) {
  c.cfg = cfg;
  CTM_HIP(hipGetDevice(&c.device));
  c.Lx = cfg.Lx; c.Ly = cfg.Ly; c.N = cfg.Lx * cfg.Ly;
  CTM_CHECK(replicas >= 1 && replicas * std::max(cfg.Lx, cfg.Ly) <= 64, -1, "context: 1..64/max(Lx, Ly) replicas");
  c.R = replicas;
  c.seeds.assign(replicas, cfg.seed);
  if (seeds) c.seeds.assign(seeds, seeds + replicas);
  c.frozen.assign(replicas, 0);
  c.failed.assign(replicas, 0);
  c.rmoves.assign(replicas, 0);
  c.layers = cfg.layers;
  c.D = cfg.D;
  c.d = (cfg.layers == 2) ? cfg.d : 1;
  c.DK = cfg.D;
  c.DB = (cfg.layers == 2) ? cfg.D : 1;
  c.Db = c.DK * c.DB;
  c.chi = cfg.chi;
  c.n = c.chi * c.Db;
  c.cutoff = (cfg.svd_rel_cutoff > 0) ? cfg.svd_rel_cutoff : 1e-12;
  const Sizes sz = sizes_of(cfg);
  const int NS = c.NS();
  c.kk = (int)sz.kk;

  if (cfg.stream) {
    c.st = (hipStream_t)cfg.stream;
  } else {
    CTM_HIP(hipStreamCreate(&c.st));
    c.own_stream = true;
  }
  c.la = linalg_create(c.st);

  // ---- site tensors and their rotations (host side, tiny) ---------------
  c.szk = (long)c.DK * c.DK * c.DK * c.DK * c.d;
  c.szb = (long)c.DB * c.DB * c.DB * c.DB * c.d;
  std::vector<double> host((size_t)NS * c.szk);
  if (on_device) {   // read on the context's stream: after the caller's prior work on it
    CTM_HIP(hipMemcpyAsync(host.data(), tensors, host.size() * sizeof(double), hipMemcpyDeviceToHost, c.st));
    CTM_HIP(hipStreamSynchronize(c.st));
  } else {
    std::memcpy(host.data(), tensors, host.size() * sizeof(double));
  }
  for (double v : host) CTM_CHECK(std::isfinite(v), -4, "site tensor has NaN/Inf entries");
  std::vector<double> ket((size_t)4 * NS * c.szk), bra((size_t)4 * NS * c.szb);
  for (int s = 0; s < NS; ++s) {
    std::vector<double> t(host.begin() + (long)s * c.szk, host.begin() + (long)(s + 1) * c.szk), r;
    for (int rot = 0; rot < 4; ++rot) {
      std::copy(t.begin(), t.end(), ket.begin() + ((long)rot * NS + s) * c.szk);
      if (c.layers == 2)
        std::copy(t.begin(), t.end(), bra.begin() + ((long)rot * NS + s) * c.szb);
      else
        bra[(long)rot * NS + s] = 1.0;
      rotate_host(t, r, c.DK, c.d);
      t.swap(r);
    }
  }
  c.Aket.alloc(ket.size() * sizeof(double));
  c.Abra.alloc(bra.size() * sizeof(double));
  CTM_HIP(hipMemcpy(c.Aket.p, ket.data(), ket.size() * sizeof(double), hipMemcpyHostToDevice));
  CTM_HIP(hipMemcpy(c.Abra.p, bra.data(), bra.size() * sizeof(double), hipMemcpyHostToDevice));

  // ---- environment ------------------------------------------------------
  const long cc = (long)c.chi * c.chi, tt = cc * c.Db;
  c.envC.alloc(sizeof(double) * 4 * NS * cc);
  c.envTa.alloc(sizeof(double) * 4 * NS * tt);
  c.envTb.alloc(sizeof(double) * 4 * NS * tt);
  std::vector<double> hb(c.Db);
  if (boundary) {
    std::memcpy(hb.data(), boundary, sizeof(double) * c.Db);
  } else if (c.layers == 2) {
    for (int a = 0; a < c.D; ++a) hb[a * c.D + a] = 1.0;
  } else {
    std::fill(hb.begin(), hb.end(), 1.0);
  }
  std::vector<double> hc(4 * NS * cc, 0.0), ht(4 * NS * tt, 0.0);
  for (int s = 0; s < 4 * NS; ++s) {
    hc[s * cc] = 1.0;
    for (int b = 0; b < c.Db; ++b) ht[s * tt + b] = hb[b];   // T[0][0][b] in the [prev][next][pair] layout
  }
  CTM_HIP(hipMemcpy(c.envC.p, hc.data(), hc.size() * sizeof(double), hipMemcpyHostToDevice));
  CTM_HIP(hipMemcpy(c.envTa.p, ht.data(), ht.size() * sizeof(double), hipMemcpyHostToDevice));
  for (int s = 0; s < NS; ++s)
    for (int k = 0; k < 4; ++k) swap_last2(c.st, c.Ta(s, k), c.Tb(s, k), c.chi, c.chi, c.Db);
  c.cdim.assign(NS, {{{1, 1}, {1, 1}, {1, 1}, {1, 1}}});
  c.tdim.assign(NS, {{{1, 1}, {1, 1}, {1, 1}, {1, 1}}});

  // ---- workspaces --------------------------------------------------------
  build_tables(c);
  const int Lmax0 = std::max(c.Lx, c.Ly) * c.R;   // cut slots of one column, all replicas
  c.Gall.alloc(sizeof(double) * 4 * sz.nn * Lmax0);                 // one slot per cut of a column
  for (int q = 0; q < 4; ++q) c.G[q].p = c.Gall.as<double>() + (size_t)q * sz.nn * Lmax0;
  c.bchunk = (int)batch_chunk(sz.nn, Lmax0);
  c.X1.alloc(sizeof(double) * c.chi * c.n * c.bchunk);
  c.X2.alloc(sizeof(double) * sz.nn * c.bchunk);
  c.ptab_words = kTableWords;
  c.ptab.alloc(sizeof(uint64_t) * c.ptab_words);
  c.ptab_host.alloc(sizeof(uint64_t) * c.ptab_words);
  c.hpin.alloc(64 << 10);
  c.ptab_used = 0;
  c.Ybuf.alloc(sizeof(double) * sz.y);
  for (auto& p : c.pan) p.alloc(sizeof(double) * c.n * c.kk * Lmax0);
  for (auto& p : c.small) p.alloc(sizeof(double) * (size_t)c.kk * c.kk * Lmax0);
  c.Svals.alloc(sizeof(double) * std::max(c.kk, c.n) * Lmax0);
  c.wvec.alloc(sizeof(double) * c.chi * Lmax0);
  if (c.kk <= kSmallLAMaxK && c.cfg.rsvd_oversample >= 0) smallla_alloc(c.sla, c.kk, Lmax0, c.n);

  c.keff.alloc(sizeof(int) * 64);
  c.badflag.alloc(sizeof(int) * c.R);   // one NaN / Inf flag per replica
  CTM_HIP(hipMemset(c.badflag.p, 0, sizeof(int) * c.R));
  c.redscratch.alloc(sizeof(double) * std::max(2048, 1025 * Lmax0));
  c.delta.alloc(sizeof(double) * c.R);
  int Lmax = Lmax0;
  c.Pt.alloc(sizeof(double) * Lmax * c.n * c.chi);
  c.PT.alloc(sizeof(double) * Lmax * c.n * c.chi);
  c.P3.alloc(sizeof(double) * Lmax * c.n * c.chi);
  c.newC1.alloc(sizeof(double) * Lmax * cc);
  c.newC4.alloc(sizeof(double) * Lmax * cc);
  c.newT4.alloc(sizeof(double) * Lmax * tt);
  c.spec.alloc(sizeof(double) * 4 * NS * c.chi);
  c.specprev.alloc(sizeof(double) * 4 * NS * c.chi);
  c.cornerscratch.alloc(sizeof(double) * 4 * NS * cc);
  c.specws.alloc(sizeof(double) * 64 + 2 * sizeof(int) * 64);
  c.gws_elems = (size_t)8 * c.n * std::max(c.kk, c.chi) * c.R;
  c.gws.alloc(sizeof(double) * c.gws_elems);
  c.amax.alloc(sizeof(unsigned) * 2);

  c.camax.alloc(sizeof(unsigned) * 4);
  switch (cfg.prec) {
    case CTM_F32: c.ctype = GemmType::F32; break;
    case CTM_BF16: c.ctype = GemmType::BF16; break;
    case CTM_F16_SPLIT: c.ctype = GemmType::F16; break;
    default: c.ctype = GemmType::F64; break;
  }
  if (uses_pre(c.cfg, c.kk)) {
    // planes per operand: hi (and lo for split FP16); the layout is the one
    // rsvd_batched addresses: [role][plane][slot][G rows, G^T rows]
    c.lp_npl = (c.ctype == GemmType::F16) ? 2 : 1;
    c.lp_ld = pre_ld(c.n);
    c.Glp.alloc(sizeof(uint16_t) * 4 * c.lp_npl * Lmax0 * 2 * c.n * c.lp_ld);
    c.panlp.alloc(sizeof(uint16_t) * c.lp_npl * Lmax0 * c.kk * c.lp_ld);
    c.panscale.alloc(sizeof(float) * Lmax0 * c.kk);
  }
  if ((c.ctype == GemmType::BF16 || c.ctype == GemmType::F16) && c.chi <= 320) {
    // the edge-corner products' operands (rows of Tp, columns of X1), per corner of a chunk
    const int npl = (c.ctype == GemmType::F16) ? 2 : 1;
    c.lp_npl = npl;
    c.x2lp.alloc(sizeof(uint16_t) * 2 * npl * c.bchunk * c.n * pre_ld(c.chi));
    c.x2rs.alloc(sizeof(float) * 2 * c.bchunk * c.n);
  }
  c.nact_cut.assign(Lmax, c.chi);
  c.cut_slot.assign(Lmax, -1);
  c.arena.first_elems = observe_arena_elems(c.chi, c.DK, c.DB, c.d);
  CTM_HIP(hipStreamSynchronize(c.st));
}

// ----------------------------------------------------------------------------
// Single-layer absorption of the site: out = X absorbed with ket then bra.
//   ket: Y[(cp,cn,r,dd)][(l',u',p)] = sum_{l,u} X[(cp,l,l')][(cn,u,u')] Ak[l][u][r][dd][p]
//   bra: out[(cn,r,r')][(cp,dd,d')] = sum_{l',u',p} Y[..][(l',u',p)] Ab[l'][u'][r'][d'][p]
//        (transposed = true: out[(cp,dd,d')][(cn,r,r')])
// ----------------------------------------------------------------------------
// GEMM on the context stream, timed under `phase` when timing is on.  The
// large contractions (edge-corner products, sketch products, projector
// formation, edge renormalisation) run in the configured precision; the GEMMs
// inside the QR / SVD of the projectors stay FP64, and so do the small
// products of the OTHER phase (C T and the corner updates: about 1% of a
// sweep's flops, where split FP16's operand scans and three MFMA passes cost
// more than FP64: 12.2 against 5.5 ms per D = 6, chi = 144 sweep).
static void mm(Context& c, int phase, int M, int N, int K, const Operand& A, const Operand& B,
               const OutOperand& C, int batch = 1) {
  const GemmType t = (phase == PhaseTimer::LINALG || phase == PhaseTimer::OTHER) ? GemmType::F64 : c.ctype;
  timed(c, phase, 2.0 * M * N * (double)K * batch, [&] {
    gemm(c.st, t, M, N, K, 1.0, A, B, 0.0, C, batch, c.ws());
  });
}

// amax (fused kernel only, nullable): receives the largest |out| (FP32 bits).
static void absorb(Context& c, const double* X, const double* Ak, const double* Ab, double* out,
                   bool transposed, unsigned* amax = nullptr) {
  const int chi = c.chi, DK = c.DK, DB = c.DB, d = c.d;
  // the fused kernel (FP64 MFMA, intermediate in registers) serves every
  // precision (an FP32-MFMA form of it measured slower: 29-30 against 26 ms
  // of absorption per D = 6, chi = 144 sweep)
  if (absorb_fused_fits(DK, DB, d)) {
    const double flops = 2.0 * chi * chi * (double)DB * DB * DK * DK * d * (DK * DK + DB * DB);
    timed(c, PhaseTimer::ABSORB, flops,
          [&] { absorb_fused(c.st, X, Ak, Ab, out, chi, DK, DB, d, transposed, amax); });
    return;
  }
  Operand A{};
  A.p = X; A.t0 = c.ketA_r.as<int>(); A.t1 = c.ketA_c.as<int>();
  Operand B = rowmajor(Ak, (long)DK * DK * d);
  OutOperand Cy{};
  Cy.p = c.Ybuf.p; Cy.t0 = c.ketC_r.as<int>(); Cy.t1 = c.ketC_c.as<int>();
  mm(c, PhaseTimer::ABSORB, chi * DB * chi * DB, DK * DK * d, DK * DK, A, B, Cy);
  Operand A2 = rowmajor(c.Ybuf.p, (long)DB * DB * d);
  Operand B2{};
  B2.p = Ab; B2.t0 = c.braB_r.as<int>(); B2.t1 = c.braB_c.as<int>();
  OutOperand Co{};
  Co.p = out;
  Co.t0 = transposed ? c.braCt_r.as<int>() : c.braCn_r.as<int>();
  Co.t1 = transposed ? c.braCt_c.as<int>() : c.braCn_c.as<int>();
  mm(c, PhaseTimer::ABSORB, chi * chi * DK * DK, DB * DB, DB * DB * d, A2, B2, Co);
}

// ---- per-problem pointer tables ---------------------------------------------
// Words are appended host-side into a blob; upload() copies the blob to the
// device ring in one stream-ordered copy and returns its device address.  The
// pinned host ring is rewritten only after the stream has drained (when the
// ring wraps), so no copy out of it can still be pending.
struct TableBlob {
  std::vector<uint64_t> w;
  void add(const void* p) { w.push_back((uint64_t)(uintptr_t)p); }
  void add_off(const double* p, const double* base) { w.push_back((uint64_t)(int64_t)(p - base)); }
};

static const uint64_t* upload(Context& c, const TableBlob& t) {
  const size_t words = t.w.size();
  CTM_CHECK(words <= c.ptab_words, -1, "pointer tables: too many problems in one launch");
  if (c.ptab_used + words > c.ptab_words) {
    CTM_HIP(hipStreamSynchronize(c.st));
    c.ptab_used = 0;
  }
  uint64_t* h = c.ptab_host.as<uint64_t>() + c.ptab_used;
  uint64_t* d = c.ptab.as<uint64_t>() + c.ptab_used;
  std::memcpy(h, t.w.data(), words * sizeof(uint64_t));
  CTM_HIP(hipMemcpyAsync(d, h, words * sizeof(uint64_t), hipMemcpyHostToDevice, c.st));
  c.ptab_used += (words + 7) & ~(size_t)7;
  return d;
}

// device views of the uploaded words
template <typename T>
static T* const* ptrs_at(const uint64_t* d, size_t i) { return reinterpret_cast<T* const*>(d + i); }
static const long* offs_at(const uint64_t* d, size_t i) { return reinterpret_cast<const long*>(d + i); }

// operands whose problem b starts at base + offs[b]
static Operand off_rowmajor(const double* base, const uint64_t* d, size_t i, long ld) {
  Operand o = rowmajor(base, ld);
  o.bo = offs_at(d, i);
  return o;
}
static Operand off_colmajor(const double* base, const uint64_t* d, size_t i, long ld) {
  Operand o = colmajor(base, ld);
  o.bo = offs_at(d, i);
  return o;
}
static OutOperand off_out_rowmajor(double* base, const uint64_t* d, size_t i, long ld) {
  OutOperand o = out_rowmajor(base, ld);
  o.bo = offs_at(d, i);
  return o;
}
static OutOperand off_out_colmajor(double* base, const uint64_t* d, size_t i, long ld) {
  OutOperand o = out_colmajor(base, ld);
  o.bo = offs_at(d, i);
  return o;
}

// X2_i = Tp_i X1_i (n x chi times chi x n, row-major) for m corners, in BF16
// or split FP16 from operands converted once per product: the rows of Tp and
// the columns of X1 become pre-converted rows (gemm_pre), so that the
// product's short K (chi) costs no conversion work per output tile.
static void x2_pre(Context& c, const std::vector<const double*>& Tp, const double* X1, long xn, double* X2, long nn) {
  const int chi = c.chi, n = c.n, m = (int)Tp.size();
  const long ldc = pre_ld(chi), obs = (long)n * ldc, lo = (long)c.bchunk * obs;
  uint16_t* Ap = c.x2lp.as<uint16_t>();
  uint16_t* Bp = Ap + (long)c.lp_npl * lo;
  float* rsA = c.x2rs.as<float>();
  float* rsB = rsA + (long)c.bchunk * n;
  timed(c, PhaseTimer::EDGE, 2.0 * n * (double)n * chi * m, [&] {
    for (int i = 0; i < m; ++i)   // row r of Tp_i (chi values) -> row r of A_i
      convert_panel_pre(c.st, c.ctype, Tp[i], 0, chi, n, 1, Ap + i * obs, obs, lo, rsA + (long)i * n, n);
    convert_cols_pre(c.st, c.ctype, X1, n, xn, chi, n, m, Bp, obs, lo, rsB, n);
    PreOperand A, B;
    A.p = Ap; A.ld = ldc; A.bs = obs; A.lo = lo; A.rowscale = rsA; A.rs_bs = n;
    B.p = Bp; B.ld = ldc; B.bs = obs; B.lo = lo; B.rowscale = rsB; B.rs_bs = n;
    gemm_pre(c.st, c.ctype, n, n, (int)ldc, 1.0, A, B, out_rowmajor(X2, n, nn), m, c.ws());
  });
}

// Enlarged corner j of site s: G[(cn, o_n)][(cp, o_p)] (n x n, row-major);
// amax (fused absorption only, nullable) receives its largest |entry|.
void enlarged_corner(Context& c, int s, int j, double* out, unsigned* amax) {
  const int chi = c.chi;
  const long n = c.n;
  // X1[tp][(cn, i_n)] = sum_t C[t][tp] Tn[t][(cn, i_n)]
  mm(c, PhaseTimer::OTHER, chi, (int)n, chi, colmajor(c.C(s, j), chi), rowmajor(c.Ta(s, j), n),
     out_rowmajor(c.X1.p, n));
  // X2[(cp, i_p)][(cn, i_n)] = sum_tp Tp[(cp, i_p)][tp] X1[tp][..]
  if (c.x2lp.p)
    x2_pre(c, {c.Tb(s, (j + 3) % 4)}, c.X1.as<double>(), (long)chi * n, c.X2.as<double>(), n * n);
  else
    mm(c, PhaseTimer::EDGE, (int)n, (int)n, chi, rowmajor(c.Tb(s, (j + 3) % 4), chi), rowmajor(c.X1.p, n),
       out_rowmajor(c.X2.p, n));
  absorb(c, c.X2.as<double>(), c.Ak(j, s), c.Ab(j, s), out, false, amax);
}

// Enlarged corners of several (site, corner, output) jobs: the same products
// as enlarged_corner, c.bchunk corners per launch (each with its own X1 / X2
// scratch), so that small corners of many cuts share their launches.
struct CornerJob {
  int s, j;
  double* out;
  unsigned* amax = nullptr;   // largest |entry| (FP32 bits, atomic max), fused absorption only
};

void enlarged_corners(Context& c, const std::vector<CornerJob>& jobs) {
  const int chi = c.chi;
  const long n = c.n, nn = n * n, xn = (long)chi * n;
  if (c.bchunk <= 1 || jobs.size() <= 1 || !absorb_fused_fits(c.DK, c.DB, c.d)) {
    for (const auto& jb : jobs) enlarged_corner(c, jb.s, jb.j, jb.out, jb.amax);
    return;
  }
  const double* envC = c.envC.as<double>();
  const double* envTa = c.envTa.as<double>();
  const double* envTb = c.envTb.as<double>();
  const double* Aket = c.Aket.as<double>();
  const double* Abra = c.Abra.as<double>();
  double* X2 = c.X2.as<double>();
  double* Gall = c.Gall.as<double>();
  for (size_t i0 = 0; i0 < jobs.size(); i0 += c.bchunk) {
    const int m = (int)std::min<size_t>(c.bchunk, jobs.size() - i0);
    const CornerJob* jb = jobs.data() + i0;
    TableBlob t;
    const size_t tC = t.w.size();
    for (int i = 0; i < m; ++i) t.add_off(c.C(jb[i].s, jb[i].j), envC);
    const size_t tTa = t.w.size();
    for (int i = 0; i < m; ++i) t.add_off(c.Ta(jb[i].s, jb[i].j), envTa);
    const size_t tTb = t.w.size();
    for (int i = 0; i < m; ++i) t.add_off(c.Tb(jb[i].s, (jb[i].j + 3) % 4), envTb);
    const size_t tX = t.w.size();
    for (int i = 0; i < m; ++i) t.add_off(X2 + i * nn, X2);
    const size_t tAk = t.w.size();
    for (int i = 0; i < m; ++i) t.add_off(c.Ak(jb[i].j, jb[i].s), Aket);
    const size_t tAb = t.w.size();
    for (int i = 0; i < m; ++i) t.add_off(c.Ab(jb[i].j, jb[i].s), Abra);
    const size_t tG = t.w.size();
    for (int i = 0; i < m; ++i) t.add_off(jb[i].out, Gall);
    const size_t tM = t.w.size();
    bool with_amax = false;
    for (int i = 0; i < m; ++i) {
      t.add(jb[i].amax);
      with_amax |= jb[i].amax != nullptr;
    }
    const uint64_t* d = upload(c, t);
    mm(c, PhaseTimer::OTHER, chi, (int)n, chi, off_colmajor(envC, d, tC, chi), off_rowmajor(envTa, d, tTa, n),
       out_rowmajor(c.X1.p, n, xn), m);
    if (c.x2lp.p) {
      std::vector<const double*> Tp(m);
      for (int i = 0; i < m; ++i) Tp[i] = c.Tb(jb[i].s, (jb[i].j + 3) % 4);
      x2_pre(c, Tp, c.X1.as<double>(), xn, X2, nn);
    } else {
      mm(c, PhaseTimer::EDGE, (int)n, (int)n, chi, off_rowmajor(envTb, d, tTb, chi), rowmajor(c.X1.p, n, xn),
         out_rowmajor(X2, n, nn), m);
    }
    const int DK = c.DK, DB = c.DB, dd = c.d;
    const double flops = 2.0 * chi * chi * (double)DB * DB * DK * DK * dd * (DK * DK + DB * DB) * m;
    timed(c, PhaseTimer::ABSORB, flops, [&] {
      absorb_fused_batched(c.st, X2, Aket, Abra, Gall, offs_at(d, tX), offs_at(d, tAk), offs_at(d, tAb),
                           offs_at(d, tG), m, chi, DK, DB, dd, false, with_amax ? ptrs_at<unsigned>(d, tM) : nullptr);
    });
  }
}

namespace {

// Y = M X with M = G_ur G_ul G_ll G_lr; panels column-major n x m.
void apply_M(Context& c, double* const G[4], const double* X, double* Y, int m, double* t1, double* t2) {
  const int n = c.n;
  // G order: 0 = UL, 1 = UR, 2 = LR, 3 = LL
  timed_group(c, PhaseTimer::SKETCH, [&] {
    mm(c, PhaseTimer::SKETCH, n, m, n, rowmajor(G[2], n), colmajor(X, n), out_colmajor(t1, n));
    mm(c, PhaseTimer::SKETCH, n, m, n, rowmajor(G[3], n), colmajor(t1, n), out_colmajor(t2, n));
    mm(c, PhaseTimer::SKETCH, n, m, n, rowmajor(G[0], n), colmajor(t2, n), out_colmajor(t1, n));
    mm(c, PhaseTimer::SKETCH, n, m, n, rowmajor(G[1], n), colmajor(t1, n), out_colmajor(Y, n));
  });
}

// Z = M^T X; W (if not null) receives G_ul^T G_ur^T X.
void apply_Mt(Context& c, double* const G[4], const double* X, double* Z, int m, double* t1, double* W) {
  const int n = c.n;
  timed_group(c, PhaseTimer::SKETCH, [&] {
    mm(c, PhaseTimer::SKETCH, n, m, n, colmajor(G[1], n), colmajor(X, n), out_colmajor(t1, n));
    mm(c, PhaseTimer::SKETCH, n, m, n, colmajor(G[0], n), colmajor(t1, n), out_colmajor(W, n));
    mm(c, PhaseTimer::SKETCH, n, m, n, colmajor(G[3], n), colmajor(W, n), out_colmajor(t1, n));
    mm(c, PhaseTimer::SKETCH, n, m, n, colmajor(G[2], n), colmajor(t1, n), out_colmajor(Z, n));
  });
}

}  // namespace

// Projectors of the cut (x, y) of a move in frame rot, into slot `slot` of
// Pt / PT (n x chi, row-major each).  Records the new bond dimension.
void cut_projectors(Context& c, int rot, int r, int x, int y, int slot) {
  const int chi = c.chi, n = c.n;
  double* Pt = c.Pt.as<double>() + (long)slot * n * chi;
  double* PT = c.PT.as<double>() + (long)slot * n * chi;
  const int o = r * c.N;
  const int sUL = o + view_site(c, rot, x, y), sUR = o + view_site(c, rot, x + 1, y);
  const int sLR = o + view_site(c, rot, x + 1, y - 1), sLL = o + view_site(c, rot, x, y - 1);
  const int nact = c.tdim[sUL][(3 + rot) % 4][0] * c.Db;
  if (nact <= chi) {   // nothing to discard: identity projectors
    identity_panel(c.st, Pt, n, chi, nact);
    identity_panel(c.st, PT, n, chi, nact);
    c.nact_cut[slot] = nact;
    c.last_cut_svd = false;
    return;
  }
  c.nact_cut[slot] = chi;
  c.last_cut_svd = true;
  // structural rank bound: smallest bond of M = G_ur G_ul G_ll G_lr (actual dims)
  int kcap = chi;
  {
    const int sites[4] = {sUL, sUR, sLR, sLL};
    for (int q = 0; q < 4; ++q) {
      const int j = (q + rot) % 4, s = sites[q];
      kcap = std::min(kcap, c.tdim[s][j][1] * c.Db);             // next leg: T_j far end
      kcap = std::min(kcap, c.tdim[s][(j + 3) % 4][0] * c.Db);   // prev leg: T_{j-1} far end
    }
  }
  double* G[4] = {c.G[0].as<double>(), c.G[1].as<double>(), c.G[2].as<double>(), c.G[3].as<double>()};
  enlarged_corner(c, sUL, (0 + rot) % 4, G[0]);
  enlarged_corner(c, sUR, (1 + rot) % 4, G[1]);
  enlarged_corner(c, sLR, (2 + rot) % 4, G[2]);
  enlarged_corner(c, sLL, (3 + rot) % 4, G[3]);
  double* P[8];
  for (int i = 0; i < 8; ++i) P[i] = c.pan[i].as<double>();
  double* S = c.Svals.as<double>();
  double* w = c.wvec.as<double>();

  if (c.cfg.rsvd_oversample < 0) {
    // exact mode: form H_u, H_d^T and M explicitly, full SVD
    double* Hu = c.X2.as<double>();
    double* HdT = c.Ybuf.as<double>();
    double* M = G[0];   // the corners are not needed once H_u and H_d^T exist
    mm(c, PhaseTimer::EDGE, n, n, n, rowmajor(G[1], n), rowmajor(G[0], n), out_rowmajor(Hu, n));
    mm(c, PhaseTimer::EDGE, n, n, n, rowmajor(G[3], n), rowmajor(G[2], n), out_rowmajor(HdT, n));
    mm(c, PhaseTimer::EDGE, n, n, n, rowmajor(Hu, n), rowmajor(HdT, n), out_colmajor(M, n));
    // M column-major: M = U S V^T directly
    double* U = P[0];
    double* VT = P[1];
    timed(c, PhaseTimer::LINALG, 0.0, [&] { la_svd(c.la, M, n, S, U, VT); });
    // V (col-major) = VT^T
    transpose_square(c.st, VT, P[2], n);
    double* V = P[2];
    projector_weights(c.st, S, U, n, n, chi, kcap, c.cutoff, w, c.keff.as<int>(), c.badflag.as<int>() + r);
    scale_columns(c.st, V, n, chi, w);
    scale_columns(c.st, U, n, chi, w);
    // Pt = H_d^T V' ; PT = H_u^T U'
    mm(c, PhaseTimer::EDGE, n, chi, n, rowmajor(HdT, n), colmajor(V, n), out_rowmajor(Pt, chi));
    mm(c, PhaseTimer::EDGE, n, chi, n, colmajor(Hu, n), colmajor(U, n), out_rowmajor(PT, chi));
    return;
  }

  const int kk = c.kk;
  double *Y = P[0], *Z = P[1], *W = P[2], *t1 = P[3], *t2 = P[4], *V = P[5], *U = P[6];
  const uint64_t sid = stream_id(c.rmoves[r], x, mod(y, (rot % 2 == 0) ? c.Ly : c.Lx));
  omega_fill(c.st, Z, n, c.Db, kk, c.seeds[r], sid);
  apply_M(c, G, Z, Y, kk, t1, t2);
  timed(c, PhaseTimer::LINALG, 0.0, [&] { la_orth(c.la, Y, n, kk); });
  for (int q = 0; q < c.cfg.rsvd_power_iters; ++q) {
    apply_Mt(c, G, Y, Z, kk, t1, W);
    timed(c, PhaseTimer::LINALG, 0.0, [&] { la_orth(c.la, Z, n, kk); });
    apply_M(c, G, Z, Y, kk, t1, t2);
    timed(c, PhaseTimer::LINALG, 0.0, [&] { la_orth(c.la, Y, n, kk); });
  }
  apply_Mt(c, G, Y, Z, kk, t1, W);                 // Z = M^T Q = B^T, W = G_ul^T G_ur^T Q
  double* R = c.small[0].as<double>();
  double* Us = c.small[1].as<double>();
  double* VTs = c.small[2].as<double>();
  timed(c, PhaseTimer::LINALG, 0.0, [&] { la_qr(c.la, Z, n, kk, R); });                         // Z <- Q2, B^T = Q2 R
  timed(c, PhaseTimer::LINALG, 0.0, [&] { la_svd(c.la, R, kk, S, Us, VTs); });                  // R = Us S VTs
  // B = R^T Q2^T = VTs^T S Us^T Q2^T  ->  Ub = VTs^T, V = Q2 Us
  mm(c, PhaseTimer::LINALG, n, kk, kk, colmajor(Z, n), colmajor(Us, kk), out_colmajor(V, n));
  // U = Q Ub, Ub(i, j) = VTs(j, i)
  mm(c, PhaseTimer::LINALG, n, kk, kk, colmajor(Y, n), rowmajor(VTs, kk), out_colmajor(U, n));
  timed(c, PhaseTimer::LINALG, 0.0, [&] {
    projector_weights(c.st, S, U, n, kk, chi, kcap, c.cutoff, w, c.keff.as<int>(), c.badflag.as<int>() + r);
  });
  scale_columns(c.st, V, n, chi, w);
  // Pt = G_ll (G_lr V')
  mm(c, PhaseTimer::EDGE, n, chi, n, rowmajor(G[2], n), colmajor(V, n), out_colmajor(t1, n));
  mm(c, PhaseTimer::EDGE, n, chi, n, rowmajor(G[3], n), colmajor(t1, n), out_rowmajor(Pt, chi));
  // PT = W Ub' with Ub'(:, i) = Ub(:, i) w_i: scale the rows of VTs first
  // (row i of VTs is column i of Ub)
  transpose_square(c.st, VTs, Us, kk);             // Us <- Ub (col-major)
  scale_columns(c.st, Us, kk, chi, w);
  mm(c, PhaseTimer::LINALG, n, chi, kk, colmajor(W, n), colmajor(Us, kk), out_rowmajor(PT, chi));
}

// Randomized-SVD projectors of the cuts of column x, batched: cut b works in
// slot s0+b of every workspace and writes Pt / PT slot s0+b.  The enlarged
// corners of all cuts are formed first (prepare); the rest runs on a range of
// the cuts, in stages that only enqueue work except for the host reads of
// stage two (the Jacobi convergence flags and the failure flags).
// Orthonormalisation by shifted Cholesky QR, the final small SVD by block
// one-sided Jacobi.  Cuts whose Cholesky factorisation was not numerically
// positive definite come back in `failed` (outputs undefined); the caller
// recomputes them with Householder QR.
struct RsvdColumn {
  Context& c;
  int rot, x, s0, nb;
  const std::vector<std::array<int, 2>>& cuts;
  int chi, n, kk;
  long nn, pk, k2, nc;
  std::vector<int> kcap;
  std::vector<uint64_t> seeds, sids;
  const unsigned* cam = nullptr;   // split FP16: per-role largest corner entry (whole column)
  bool pre = false;                // reduced-type corner and panel operands
  int npl = 1;
  long ld = 0, gobs = 0, glo = 0, pobs = 0, plo = 0;

  RsvdColumn(Context& cc, int rot_, int x_, const std::vector<std::array<int, 2>>& cuts_, int s0_)
      : c(cc), rot(rot_), x(x_), s0(s0_), nb((int)cuts_.size()), cuts(cuts_), chi(cc.chi), n(cc.n), kk(cc.kk) {
    nn = (long)n * n; pk = (long)n * kk; k2 = (long)kk * kk; nc = (long)n * chi;
  }
  double* Gp(int role, int slot) const { return c.G[role].as<double>() + slot * nn; }
  double* pan(int i, int slot) const { return c.pan[i].as<double>() + slot * pk; }
  uint16_t* Glp(int role, int slot) const {
    return c.Glp.as<uint16_t>() + (long)role * npl * glo + slot * gobs;
  }

  // Enlarged corners, sketch seeds and operand scales of every cut (c.st).
  void prepare() {
    kcap.assign(nb, chi);
    seeds.assign(nb, 0);
    sids.assign(nb, 0);
    std::vector<CornerJob> jobs;
    // split FP16: each corner role's largest entry over the column, from the
    // absorption that forms the corners (or a scan when it is not fused)
    const bool f16 = c.ctype == GemmType::F16;
    const bool fused = absorb_fused_fits(c.DK, c.DB, c.d);
    unsigned* camax = c.camax.as<unsigned>();
    if (f16 && fused) clear_words(c.st, camax, 4);
    for (int b = 0; b < nb; ++b) {
      const int r = cuts[b][0], y = cuts[b][1], slot = s0 + b, o = r * c.N;
      const int sites[4] = {o + view_site(c, rot, x, y), o + view_site(c, rot, x + 1, y),
                            o + view_site(c, rot, x + 1, y - 1), o + view_site(c, rot, x, y - 1)};
      for (int q = 0; q < 4; ++q) {
        const int j = (q + rot) % 4, s = sites[q];
        kcap[b] = std::min(kcap[b], c.tdim[s][j][1] * c.Db);
        kcap[b] = std::min(kcap[b], c.tdim[s][(j + 3) % 4][0] * c.Db);
        jobs.push_back({s, j, Gp(q, slot), (f16 && fused) ? camax + q : nullptr});   // roles: 0 UL, 1 UR, 2 LR, 3 LL
      }
      seeds[b] = c.seeds[r];
      sids[b] = stream_id(c.rmoves[r], x, y);
    }
    enlarged_corners(c, jobs);
    if (f16) {
      if (!fused)
        for (int role = 0; role < 4; ++role)
          operand_amax(c.st, rowmajor(Gp(role, s0), n, nn), n, n, nb, camax + role);
      cam = camax;
    }
    // BF16 / split FP16: every corner (and its transpose) converted once per
    // column, every panel once per product
    pre = c.Glp.p != nullptr && (c.ctype == GemmType::BF16 || c.ctype == GemmType::F16);
    npl = c.lp_npl;
    CTM_CHECK(!pre || npl == (c.ctype == GemmType::F16 ? 2 : 1), -1, "reduced-type corner planes");
    const long Lslots = std::max(c.Lx, c.Ly) * (long)c.R;
    ld = c.lp_ld;
    gobs = 2L * n * ld; glo = Lslots * gobs; pobs = (long)kk * ld; plo = Lslots * pobs;
    if (pre)
      timed(c, PhaseTimer::SKETCH, 0.0, [&] {
        for (int role = 0; role < 4; ++role)
          convert_square_pre(c.st, c.ctype, Gp(role, s0), nn, n, nb, Glp(role, s0), gobs, glo,
                             cam ? cam + role : nullptr);
      });
  }

  // ---- products of cuts [b0, b1) ----------------------------------------
  // A (n x n, G or G^T) times the panel X (n x m, column-major) -> out
  void pre_prod(int b0, int b1, int phase, int role, bool trans, const double* X, int m, const OutOperand& out) {
    const int sb = s0 + b0, nbh = b1 - b0;
    timed(c, phase, 2.0 * n * m * (double)n * nbh, [&] {
      float* rs = c.panscale.as<float>() + (long)sb * kk;
      uint16_t* xp = c.panlp.as<uint16_t>() + sb * pobs;
      convert_panel_pre(c.st, c.ctype, X, pk, n, m, nbh, xp, pobs, plo, rs, kk);
      PreOperand A, B;
      A.p = Glp(role, sb) + (trans ? (long)n * ld : 0);
      A.ld = ld; A.bs = gobs; A.lo = glo; A.amax = cam ? cam + role : nullptr;
      B.p = xp; B.ld = ld; B.bs = pobs; B.lo = plo; B.rowscale = rs; B.rs_bs = kk;
      gemm_pre(c.st, c.ctype, n, m, (int)ld, 1.0, A, B, out, nbh, c.ws());
    });
  }
  void prod(int b0, int b1, int role, bool trans, const double* X, double* Yo, int m) {
    if (pre) {
      pre_prod(b0, b1, PhaseTimer::SKETCH, role, trans, X, m, out_colmajor(Yo, n, pk));
      return;
    }
    const int sb = s0 + b0;
    Operand A = trans ? colmajor(Gp(role, sb), n, nn) : rowmajor(Gp(role, sb), n, nn);
    if (cam) A.amax = cam + role;
    mm(c, PhaseTimer::SKETCH, n, m, n, A, colmajor(X, n, pk), out_colmajor(Yo, n, pk), b1 - b0);
  }
  // Yo = G_ur G_ul G_ll G_lr X
  void applyM(int b0, int b1, const double* X, double* Yo) {
    double *t1 = pan(3, s0 + b0), *t2 = pan(4, s0 + b0);
    timed_group(c, PhaseTimer::SKETCH, [&] {
      prod(b0, b1, 2, false, X, t1, kk); prod(b0, b1, 3, false, t1, t2, kk);
      prod(b0, b1, 0, false, t2, t1, kk); prod(b0, b1, 1, false, t1, Yo, kk);
    });
  }
  // Zo = M^T X, W = G_ul^T G_ur^T X
  void applyMt(int b0, int b1, const double* X, double* Zo) {
    double *t1 = pan(3, s0 + b0), *W = pan(2, s0 + b0);
    timed_group(c, PhaseTimer::SKETCH, [&] {
      prod(b0, b1, 1, true, X, t1, kk); prod(b0, b1, 0, true, t1, W, kk);
      prod(b0, b1, 3, true, W, t1, kk); prod(b0, b1, 2, true, t1, Zo, kk);
    });
  }
  void orth(int b0, int b1, double* P, int passes, double* Racc) {
    timed(c, PhaseTimer::LINALG, 0.0, [&] { cholqr(c.st, c.sla, P, pk, n, kk, b1 - b0, passes, Racc, c.ws()); });
  }

  // Stage 1a: the sketch matrix and the first range product Y = M Omega.
  void stage1a(int b0, int b1) {
    const int sb = s0 + b0, nbh = b1 - b0;
    timed(c, PhaseTimer::OTHER, 0.0, [&] {
      omega_fill_batched(c.st, pan(1, sb), pk, nbh, n, c.Db, kk, seeds.data() + b0, sids.data() + b0);
    });
    applyM(b0, b1, pan(1, sb), pan(0, sb));
  }
  // Stage 1b: power iterations, B^T = M^T Q = Q2 R, and the Jacobi sweeps
  // that run before the first convergence read.  Intermediate bases need
  // unit-norm directions but not full orthogonality: the shifted pass alone
  // damps every direction below the shift (so power iterations would lose
  // the small kept singular values), the second pass restores the norms.
  // The final basis takes a third pass.
  void stage1b(int b0, int b1) {
    const int sb = s0 + b0, nbh = b1 - b0;
    double *Y = pan(0, sb), *Z = pan(1, sb);
    const int q = c.cfg.rsvd_power_iters;
    orth(b0, b1, Y, q == 0 ? 3 : 2, nullptr);
    for (int it = 0; it < q; ++it) {
      applyMt(b0, b1, Y, Z);
      orth(b0, b1, Z, 2, nullptr);
      applyM(b0, b1, Z, Y);
      orth(b0, b1, Y, it == q - 1 ? 3 : 2, nullptr);
    }
    applyMt(b0, b1, Y, Z);                           // Z = M^T Q = B^T
    double* R = c.small[0].as<double>() + sb * k2;
    orth(b0, b1, Z, 3, R);                           // Z <- Q2, B^T = Q2 R
    // R = X diag(S) Ysv^T  ->  B = Ysv S (Q2 X)^T : Ub = Ysv, V = Q2 X.
    // The one-sided Jacobi runs on R^T = Ysv S X^T, whose rows are graded
    // like the sketch directions, and converges in fewer sweeps than on R.
    double* Rt = c.small[3].as<double>() + sb * k2;
    timed(c, PhaseTimer::LINALG, 0.0, [&] {
      transpose_square_batched(c.st, R, Rt, kk, nbh);
      jacobi_svd_start(c.st, c.sla, Rt, kk, nbh);
    });
  }
  // Stage 2: the rest of the Jacobi, the projectors, and the flags (host
  // reads on c.st).  failed: indices b in [b0, b1).
  void stage2(int b0, int b1, std::vector<int>& failed) {
    const int sb = s0 + b0, nbh = b1 - b0;
    double *Y = pan(0, sb), *Z = pan(1, sb), *W = pan(2, sb), *t1 = pan(3, sb);
    double *V = pan(5, sb), *U = pan(6, sb);
    double* X = c.small[1].as<double>() + sb * k2;
    double* Ysv = c.small[2].as<double>() + sb * k2;
    double* Rt = c.small[3].as<double>() + sb * k2;
    double* S = c.Svals.as<double>() + (long)sb * std::max(kk, n);
    timed(c, PhaseTimer::LINALG, 0.0, [&] { jacobi_svd_finish(c.st, c.sla, Rt, kk, nbh, Ysv, S, std::max(kk, n), X); });
    mm(c, PhaseTimer::LINALG, n, kk, kk, colmajor(Z, n, pk), colmajor(X, kk, k2), out_colmajor(V, n, pk), nbh);
    mm(c, PhaseTimer::LINALG, n, kk, kk, colmajor(Y, n, pk), colmajor(Ysv, kk, k2), out_colmajor(U, n, pk), nbh);
    {
      double* w = c.wvec.as<double>() + (long)sb * chi;
      timed(c, PhaseTimer::LINALG, 0.0, [&] {
        projector_weights_batched(c.st, S, std::max(kk, n), U, pk, n, kk, chi, kcap.data() + b0, c.cutoff, w,
                                  c.keff.as<int>() + sb, c.sla.flag.as<int>() + 128, nbh);
        scale_columns_batched(c.st, V, pk, nbh, n, chi, w, chi);
        scale_columns_batched(c.st, Ysv, k2, nbh, kk, chi, w, chi);
      });
    }
    // Pt = G_ll (G_lr V'), PT = W Ub'
    double* Pt = c.Pt.as<double>() + sb * nc;
    double* PT = c.PT.as<double>() + sb * nc;
    if (pre) {
      pre_prod(b0, b1, PhaseTimer::EDGE, 2, false, V, chi, out_colmajor(t1, n, pk));
      pre_prod(b0, b1, PhaseTimer::EDGE, 3, false, t1, chi, out_rowmajor(Pt, chi, nc));
    } else {
      Operand G2 = rowmajor(Gp(2, sb), n, nn), G3 = rowmajor(Gp(3, sb), n, nn);
      if (cam) {
        G2.amax = cam + 2;
        G3.amax = cam + 3;
      }
      mm(c, PhaseTimer::EDGE, n, chi, n, G2, colmajor(V, n, pk), out_colmajor(t1, n, pk), nbh);
      mm(c, PhaseTimer::EDGE, n, chi, n, G3, colmajor(t1, n, pk), out_rowmajor(Pt, chi, nc), nbh);
    }
    mm(c, PhaseTimer::LINALG, n, chi, kk, colmajor(W, n, pk), colmajor(Ysv, kk, k2), out_rowmajor(PT, chi, nc), nbh);
    // cuts whose Cholesky QR broke down
    int flags[192] = {0};
    d2h(c, flags, c.sla.flag.as<int>(), 192);
    bool any = false, numeric = false;
    for (int b = 0; b < nbh; ++b) {
      if (flags[b]) {
        failed.push_back(b0 + b);
      } else if (flags[128 + b]) {   // no singular value above zero
        numeric = true;
        c.failed[cuts[b0 + b][0]] = 1;
      }
      any |= flags[b] || flags[128 + b];
    }
    if (any) {
      CTM_HIP(hipMemsetAsync(c.sla.flag.p, 0, sizeof(int) * 64, c.st));
      CTM_HIP(hipMemsetAsync(c.sla.flag.as<int>() + 128, 0, sizeof(int) * 64, c.st));
    }
    if (g_debug) {
      fprintf(stderr, "[ctm] move %lld rot %d col %d slots %d..%d: cholqr codes", c.moves, rot, x, sb, sb + nbh - 1);
      for (int b = 0; b < nbh; ++b) fprintf(stderr, " %d", flags[b]);
      fprintf(stderr, "\n");
    }
    if (numeric && !c.isolate) {
      for (int b = b0; b < b1; ++b) c.failed[cuts[b][0]] = 0;
      throw Error(-4, "projectors: a cut has no singular value above zero");
    }
  }
};

static void rsvd_batched(Context& c, int rot, int x, const std::vector<std::array<int, 2>>& cuts, int s0,
                         std::vector<int>& failed) {
  RsvdColumn col(c, rot, x, cuts, s0);
  failed.clear();
  col.prepare();
  col.stage1a(0, col.nb);
  col.stage1b(0, col.nb);
  col.stage2(0, col.nb, failed);
}

// Projectors of every cut of column x of every live replica (identity,
// batched randomized SVD, or the Householder / exact-SVD path).  Cut (r, y)
// gets slot cut_slot[r * Lyv + y]: the live cuts numbered in order.
static void column_projectors(Context& c, int rot, int x, int Lyv) {
  std::vector<std::array<int, 2>> svd;
  std::vector<int> svd_slot;
  int slot = 0;
  for (int r = 0; r < c.R; ++r)
    for (int y = 0; y < Lyv; ++y) {
      if (c.frozen[r]) {
        c.cut_slot[r * Lyv + y] = -1;
        continue;
      }
      c.cut_slot[r * Lyv + y] = slot;
      const int nact = c.tdim[r * c.N + view_site(c, rot, x, y)][(3 + rot) % 4][0] * c.Db;
      if (nact <= c.chi) {
        cut_projectors(c, rot, r, x, y, slot);   // identity
        ++c.cuts[0];
      } else {
        svd.push_back({r, y});
        svd_slot.push_back(slot);
      }
      ++slot;
    }
  if (svd.empty()) return;
  const bool fast = c.cfg.rsvd_oversample >= 0 && c.cfg.projector_path == CTM_PATH_AUTO && c.sla.kmax > 0 &&
                    smallla_fits(c.sla, c.kk);
  if (!fast) {
    for (size_t i = 0; i < svd.size(); ++i) cut_projectors(c, rot, svd[i][0], x, svd[i][1], svd_slot[i]);
    c.cuts[2] += (int64_t)svd.size();
    return;
  }
  std::vector<int> failed;
  auto run = [&](const std::vector<std::array<int, 2>>& cuts, int s0) {
    rsvd_batched(c, rot, x, cuts, s0, failed);
    for (int b : failed) cut_projectors(c, rot, cuts[b][0], x, cuts[b][1], s0 + b);   // Householder fallback
    for (int b = 0; b < (int)cuts.size(); ++b) c.nact_cut[s0 + b] = c.chi;
    c.cuts[1] += (int64_t)cuts.size() - (int64_t)failed.size();
    c.cuts[2] += (int64_t)failed.size();
  };
  if ((int)svd.size() == slot) {
    run(svd, 0);   // every live cut: one batch over contiguous slots
  } else {
    for (size_t i = 0; i < svd.size(); ++i) run({svd[i]}, svd_slot[i]);
  }
  c.last_cut_svd = true;
}

// Single cut through the same path as a move (used by ctm_projectors); slot 0.
void cut_projectors_fast(Context& c, int rot, int x, int y) {
  const int nact = c.tdim[view_site(c, rot, x, y)][(3 + rot) % 4][0] * c.Db;
  if (nact <= c.chi || c.cfg.rsvd_oversample < 0 || c.cfg.projector_path != CTM_PATH_AUTO || c.sla.kmax == 0 ||
      !smallla_fits(c.sla, c.kk)) {
    cut_projectors(c, rot, 0, x, y, 0);
    ++c.cuts[nact <= c.chi ? 0 : 2];
    return;
  }
  std::vector<int> failed;
  rsvd_batched(c, rot, x, {{0, y}}, 0, failed);
  if (!failed.empty()) cut_projectors(c, rot, 0, x, y, 0);
  ++c.cuts[failed.empty() ? 1 : 2];
  c.nact_cut[0] = c.chi;
  c.last_cut_svd = true;
}

// Pointers of one cut's column update (see do_move).
struct UpdPtrs {
  int s = 0, r = 0;   // old site, replica
  double *Pt_up = nullptr, *Pt_dn = nullptr, *PT_dn = nullptr, *PT_up = nullptr, *P3_up = nullptr;
  double *C1n = nullptr, *C4n = nullptr, *T4n = nullptr;
};

// The column update of do_move for `count` cuts, c.bchunk cuts per launch:
// every launch runs one step of the per-cut sequence for all cuts of the
// chunk, each with its own X1, X2 and G[0] scratch, so each cut gets exactly
// the arithmetic of the per-cut sequence.  fill(i, ptrs) describes cut i.
template <typename F>
static void update_column_batched(Context& c, int rot, bool direct, size_t count, F&& fill) {
  const int chi = c.chi, Db = c.Db;
  const long n = c.n, nn = n * n, cc = (long)chi * chi, tt = cc * Db, xn = (long)chi * n;
  const int kc1 = rot % 4, kt1 = rot % 4, kt3 = (2 + rot) % 4, kt4 = (3 + rot) % 4, kc4 = (3 + rot) % 4;
  double* X1 = c.X1.as<double>();
  double* X2 = c.X2.as<double>();
  double* G0 = c.G[0].as<double>();
  double* envC = c.envC.as<double>();
  double* envTa = c.envTa.as<double>();
  const double* envTb = c.envTb.as<double>();
  const double* Pt = c.Pt.as<double>();
  const double* PT = c.PT.as<double>();
  const double* P3 = c.P3.as<double>();
  const double* Aket = c.Aket.as<double>();
  const double* Abra = c.Abra.as<double>();
  // where the new tensors go (see do_move)
  double* C1base = direct ? envC : c.newC1.as<double>();
  double* C4base = direct ? envC : c.newC4.as<double>();
  double* T4base = direct ? envTa : c.newT4.as<double>();
  for (size_t i0 = 0; i0 < count; i0 += c.bchunk) {
    const int m = (int)std::min<size_t>(c.bchunk, count - i0);
    std::vector<UpdPtrs> q(m);
    for (int i = 0; i < m; ++i) fill(i0 + i, q[i]);
    TableBlob t;
    auto each = [&](auto get) {   // m entries
      const size_t at = t.w.size();
      for (int i = 0; i < m; ++i) get(i);
      return at;
    };
    auto each_inner = [&](auto get) {   // m * chi entries, problem i * chi + k
      const size_t at = t.w.size();
      for (int i = 0; i < m; ++i)
        for (int k = 0; k < chi; ++k) get(i, k);
      return at;
    };
    // pointer tables (edge transposes, normalisation)
    const size_t pPTup = each([&](int i) { t.add(q[i].PT_up); });
    const size_t pP3up = each([&](int i) { t.add(q[i].P3_up); });
    const size_t pC1n = each([&](int i) { t.add(q[i].C1n); });
    const size_t pC4n = each([&](int i) { t.add(q[i].C4n); });
    const size_t pT4n = each([&](int i) { t.add(q[i].T4n); });
    // offset tables (GEMM, absorption)
    const size_t oA1 = each_inner([&](int i, int) { t.add_off(c.C(q[i].s, kc1), envC); });
    const size_t oB1 = each_inner([&](int i, int k) { t.add_off(c.Ta(q[i].s, kt1) + (long)k * Db, envTa); });
    const size_t oX1 = each_inner([&](int i, int k) { t.add_off(X1 + i * xn + (long)k * chi * Db, X1); });
    const size_t oPtup = each([&](int i) { t.add_off(q[i].Pt_up, Pt); });
    const size_t oC1n = each([&](int i) { t.add_off(q[i].C1n, C1base); });
    const size_t oA4 = each_inner([&](int i, int) { t.add_off(c.C(q[i].s, kc4), envC); });
    const size_t oB4 = each_inner([&](int i, int k) { t.add_off(c.Ta(q[i].s, kt3) + (long)k * chi * Db, envTa); });
    const size_t oPTdn = each([&](int i) { t.add_off(q[i].PT_dn, PT); });
    const size_t oC4n = each([&](int i) { t.add_off(q[i].C4n, C4base); });
    const size_t oTb = each([&](int i) { t.add_off(c.Tb(q[i].s, kt4), envTb); });
    const size_t oP3up = each([&](int i) { t.add_off(q[i].P3_up, P3); });
    const size_t oX2 = each([&](int i) { t.add_off(X2 + i * nn, X2); });
    const size_t oAk = each([&](int i) { t.add_off(c.Ak(rot, q[i].s), Aket); });
    const size_t oAb = each([&](int i) { t.add_off(c.Ab(rot, q[i].s), Abra); });
    const size_t oG0 = each([&](int i) { t.add_off(G0 + i * nn, G0); });
    const size_t oPtdn = each([&](int i) { t.add_off(q[i].Pt_dn, Pt); });
    const size_t oT4n = each([&](int i) { t.add_off(q[i].T4n, T4base); });
    const size_t oRep = each([&](int i) { t.w.push_back((uint64_t)q[i].r); });   // failure flag of each cut
    const uint64_t* d = upload(c, t);
    swap_last2_batched(c.st, ptrs_at<const double>(d, pPTup), ptrs_at<double>(d, pP3up), m, chi, Db, chi);
    // C1' = (C1 T1) Pt_up
    mm(c, PhaseTimer::OTHER, chi, Db, chi, off_colmajor(envC, d, oA1, chi), off_rowmajor(envTa, d, oB1, n),
       off_out_rowmajor(X1, d, oX1, Db), m * chi);
    mm(c, PhaseTimer::OTHER, chi, chi, (int)n, rowmajor(X1, n, xn), off_rowmajor(Pt, d, oPtup, chi),
       off_out_rowmajor(C1base, d, oC1n, chi), m);
    // C4'^T = (C4 T3) PT_dn
    mm(c, PhaseTimer::OTHER, chi, Db, chi, off_rowmajor(envC, d, oA4, chi), off_rowmajor(envTa, d, oB4, Db),
       off_out_rowmajor(X1, d, oX1, Db), m * chi);
    mm(c, PhaseTimer::OTHER, chi, chi, (int)n, rowmajor(X1, n, xn), off_rowmajor(PT, d, oPTdn, chi),
       off_out_colmajor(C4base, d, oC4n, chi), m);
    // T4' = Pt_dn^T absorb(T4 P3_up)
    mm(c, PhaseTimer::EDGE, (int)n, (int)n, chi, off_rowmajor(envTb, d, oTb, chi), off_rowmajor(P3, d, oP3up, n),
       out_rowmajor(X2, n, nn), m);
    const int DK = c.DK, DB = c.DB, dd = c.d;
    const double flops = 2.0 * chi * chi * (double)DB * DB * DK * DK * dd * (DK * DK + DB * DB) * m;
    timed(c, PhaseTimer::ABSORB, flops, [&] {
      absorb_fused_batched(c.st, X2, Aket, Abra, G0, offs_at(d, oX2), offs_at(d, oAk), offs_at(d, oAb),
                           offs_at(d, oG0), m, chi, DK, DB, dd, true);
    });
    mm(c, PhaseTimer::EDGE, chi, (int)n, (int)n, off_colmajor(Pt, d, oPtdn, chi), rowmajor(G0, n, nn),
       off_out_rowmajor(T4base, d, oT4n, n), m);
    int* bad = c.badflag.as<int>();
    normalize_maxabs_batched(c.st, ptrs_at<double>(d, pC1n), m, cc, c.redscratch.as<double>(), bad, offs_at(d, oRep));
    normalize_maxabs_batched(c.st, ptrs_at<double>(d, pC4n), m, cc, c.redscratch.as<double>(), bad, offs_at(d, oRep));
    normalize_maxabs_batched(c.st, ptrs_at<double>(d, pT4n), m, tt, c.redscratch.as<double>(), bad, offs_at(d, oRep));
  }
}

// One directional move (Sec. 2.2) in the frame rotated rot quarter turns, for
// every live replica.
void do_move(Context& c, int rot) {
  int Lxv, Lyv;
  view_dims(c, rot, Lxv, Lyv);
  const int chi = c.chi, n = c.n, Db = c.Db;
  const long cc = (long)chi * chi, tt = cc * Db;
  const int kc1 = (0 + rot) % 4, kt1 = (0 + rot) % 4, kt3 = (2 + rot) % 4, kt4 = (3 + rot) % 4, kc4 = (3 + rot) % 4;
  const bool direct = Lxv > 1;
  for (int x = 0; x < Lxv; ++x) {
    column_projectors(c, rot, x, Lyv);
    std::vector<std::array<int, 2>> newdC1(c.R * Lyv), newdT4(c.R * Lyv), newdC4(c.R * Lyv);
    // the live cuts of the column: old site s, new site t, own slot, slot above
    struct Upd { int ry, s, t, sl, up; };
    std::vector<Upd> ups;
    for (int r = 0; r < c.R; ++r) {
      if (c.frozen[r]) continue;
      for (int y = 0; y < Lyv; ++y)
        ups.push_back({r * Lyv + y, r * c.N + view_site(c, rot, x, y), r * c.N + view_site(c, rot, x + 1, y),
                       c.cut_slot[r * Lyv + y], c.cut_slot[r * Lyv + (y + 1) % Lyv]});
    }
    // the new tensors go to column x + 1; with one column they replace
    // tensors other cuts still read, so they are staged first
    auto C1n_of = [&](const Upd& u) { return direct ? c.C(u.t, kc1) : c.newC1.as<double>() + u.sl * cc; };
    auto C4n_of = [&](const Upd& u) { return direct ? c.C(u.t, kc4) : c.newC4.as<double>() + u.sl * cc; };
    auto T4n_of = [&](const Upd& u) { return direct ? c.Ta(u.t, kt4) : c.newT4.as<double>() + u.sl * tt; };
    const bool batched = c.bchunk > 1 && ups.size() > 1 && absorb_fused_fits(c.DK, c.DB, c.d);
    if (batched) {
      update_column_batched(c, rot, direct, ups.size(), [&](size_t i, UpdPtrs& q) {
        const Upd& u = ups[i];
        q.s = u.s;
        q.r = u.ry / Lyv;
        q.Pt_up = c.Pt.as<double>() + (long)u.up * n * chi;
        q.Pt_dn = c.Pt.as<double>() + (long)u.sl * n * chi;
        q.PT_dn = c.PT.as<double>() + (long)u.sl * n * chi;
        q.PT_up = c.PT.as<double>() + (long)u.up * n * chi;
        q.P3_up = c.P3.as<double>() + (long)u.up * n * chi;
        q.C1n = C1n_of(u);
        q.C4n = C4n_of(u);
        q.T4n = T4n_of(u);
      });
    }
    for (const Upd& u : ups) {
      const int s = u.s, sl = u.sl, up = u.up;
      if (!batched) {
        double* Pt_up = c.Pt.as<double>() + (long)up * n * chi;
        double* Pt_dn = c.Pt.as<double>() + (long)sl * n * chi;
        double* PT_dn = c.PT.as<double>() + (long)sl * n * chi;
        double* P3_up = c.P3.as<double>() + (long)up * n * chi;
        swap_last2(c.st, c.PT.as<double>() + (long)up * n * chi, P3_up, chi, Db, chi);
        double* C1n = C1n_of(u);
        double* C4n = C4n_of(u);
        double* T4n = T4n_of(u);
        // C1' = (C1 T1) Pt_up: X1p[c2][(t4, u)] then times Pt
        mm(c, PhaseTimer::OTHER, chi, Db, chi, colmajor(c.C(s, kc1), chi), rowmajor(c.Ta(s, kt1), n, Db),
           out_rowmajor(c.X1.p, Db, (long)chi * Db), chi);
        mm(c, PhaseTimer::OTHER, chi, chi, n, rowmajor(c.X1.p, n), rowmajor(Pt_up, chi), out_rowmajor(C1n, chi));
        // C4'^T[c3][k] = sum_{(t4,d)} Yc[c3][(t4, d)] PT_dn[(t4, d)][k], Yc[c3] = C4 T3[c3]
        mm(c, PhaseTimer::OTHER, chi, Db, chi, rowmajor(c.C(s, kc4), chi),
           rowmajor(c.Ta(s, kt3), Db, (long)chi * Db), out_rowmajor(c.X1.p, Db, (long)chi * Db), chi);
        mm(c, PhaseTimer::OTHER, chi, chi, n, rowmajor(c.X1.p, n), rowmajor(PT_dn, chi), out_colmajor(C4n, chi));
        // T4' = Pt_dn^T absorb(T4 P3_up)
        if (c.x2lp.p)
          x2_pre(c, {c.Tb(s, kt4)}, P3_up, (long)chi * n, c.X2.as<double>(), (long)n * n);
        else
          mm(c, PhaseTimer::EDGE, n, n, chi, rowmajor(c.Tb(s, kt4), chi), rowmajor(P3_up, n),
             out_rowmajor(c.X2.p, n));
        // split FP16: the absorption also returns the largest |G0|, the scale
        // source of the product that follows (no scan of G0)
        unsigned* g0max = nullptr;
        if (c.ctype == GemmType::F16 && absorb_fused_fits(c.DK, c.DB, c.d)) {
          g0max = c.camax.as<unsigned>();
          clear_words(c.st, g0max, 1);
        }
        absorb(c, c.X2.as<double>(), c.Ak(rot, s), c.Ab(rot, s), c.G[0].as<double>(), true, g0max);
        Operand G0op = rowmajor(c.G[0].p, n);
        G0op.amax = g0max;
        mm(c, PhaseTimer::EDGE, chi, n, n, colmajor(Pt_dn, chi), G0op, out_rowmajor(T4n, n));
        int* bad = c.badflag.as<int>() + u.ry / Lyv;
        normalize_maxabs(c.st, C1n, cc, c.redscratch.as<double>(), bad);
        normalize_maxabs(c.st, C4n, cc, c.redscratch.as<double>(), bad);
        normalize_maxabs(c.st, T4n, tt, c.redscratch.as<double>(), bad);
      }
      newdC1[u.ry] = {c.tdim[s][kt1][1], c.nact_cut[up]};
      newdT4[u.ry] = {c.nact_cut[sl], c.nact_cut[up]};
      newdC4[u.ry] = {c.nact_cut[sl], c.tdim[s][kt3][0]};
    }
    std::vector<double*> swaps_in, swaps_out;   // batched: Ta -> Tb of the new edges
    for (int r = 0; r < c.R; ++r) {
      if (c.frozen[r]) continue;
      for (int y = 0; y < Lyv; ++y) {
        const int t = r * c.N + view_site(c, rot, x + 1, y), sl = c.cut_slot[r * Lyv + y];
        if (!direct) {
          CTM_HIP(hipMemcpyAsync(c.C(t, kc1), c.newC1.as<double>() + sl * cc, cc * sizeof(double),
                                 hipMemcpyDeviceToDevice, c.st));
          CTM_HIP(hipMemcpyAsync(c.C(t, kc4), c.newC4.as<double>() + sl * cc, cc * sizeof(double),
                                 hipMemcpyDeviceToDevice, c.st));
          CTM_HIP(hipMemcpyAsync(c.Ta(t, kt4), c.newT4.as<double>() + sl * tt, tt * sizeof(double),
                                 hipMemcpyDeviceToDevice, c.st));
        }
        if (batched) {
          swaps_in.push_back(c.Ta(t, kt4));
          swaps_out.push_back(c.Tb(t, kt4));
        } else {
          swap_last2(c.st, c.Ta(t, kt4), c.Tb(t, kt4), chi, chi, Db);
        }
        c.cdim[t][kc1] = newdC1[r * Lyv + y];
        c.tdim[t][kt4] = newdT4[r * Lyv + y];
        c.cdim[t][kc4] = newdC4[r * Lyv + y];
      }
    }
    if (!swaps_in.empty()) {
      TableBlob sw;
      for (double* p : swaps_in) sw.add(p);
      for (double* p : swaps_out) sw.add(p);
      const uint64_t* d = upload(c, sw);
      swap_last2_batched(c.st, ptrs_at<const double>(d, 0), ptrs_at<double>(d, swaps_in.size()), (int)swaps_in.size(),
                         chi, chi, Db);
    }
  }
  for (int r = 0; r < c.R; ++r)
    if (!c.frozen[r]) c.rmoves[r] += 1;
  c.moves += 1;
  check_bad(c, "ctm_move");
}

static const int kSweepRot[4] = {0, 2, 1, 3};   // left, right, up, down

static void corner_spectra(Context& c, double* out) {
  const long cc = (long)c.chi * c.chi;
  timed(c, PhaseTimer::OTHER, 0.0, [&] {
    if (c.chi <= kSvSmallMax) {   // one workgroup per corner, the corners read in place
      singular_values_small(c.st, c.envC.as<double>(), c.chi, 4 * c.NS(), out);
      return;
    }
    CTM_HIP(hipMemcpyAsync(c.cornerscratch.p, c.envC.p, sizeof(double) * 4 * c.NS() * cc, hipMemcpyDeviceToDevice,
                           c.st));
    for (int i = 0; i < 4 * c.NS(); i += 64) {
      const int nb = std::min(64, 4 * c.NS() - i);
      double* A = c.cornerscratch.as<double>() + i * cc;
      if (c.chi <= kSmallLAMaxK) {   // blocked one-sided Jacobi, values only (C^T: same values)
        double* off = c.specws.as<double>();
        int* conv = reinterpret_cast<int*>(off + 64);
        singular_values_batched(c.st, A, c.chi, nb, out + (long)i * c.chi, c.chi, off, conv, conv + 64,
                                c.hpin.as<int>());
      } else {
        la_singular_values_batched(c.la, A, c.chi, nb, out + (long)i * c.chi);
      }
    }
  });
}

// delta of every replica (device, c.delta[r]): spectra of the 4 N corners of
// replica r against their previous values; prev <- spectra.
static void replica_deltas(Context& c, double* spec, double* prev) {
  const long per = 4L * c.N * c.chi;
  for (int r = 0; r < c.R; ++r)
    spectra_delta(c.st, spec + r * per, prev + r * per, 4 * c.N, c.chi, c.delta.as<double>() + r);
}

void group_start(Context& c) {
  corner_spectra(c, c.specprev.as<double>());
  // normalise the reference spectra (deltas of this step are discarded)
  replica_deltas(c, c.specprev.as<double>(), c.spec.as<double>());
  CTM_HIP(hipMemcpyAsync(c.specprev.p, c.spec.p, sizeof(double) * 4 * c.NS() * c.chi, hipMemcpyDeviceToDevice,
                         c.st));
}

void group_sweep(Context& c, double* host_delta) {
  for (int m = 0; m < 4; ++m) {
    do_move(c, kSweepRot[m]);
    // a replica that failed in this move takes no further moves
    for (int r = 0; r < c.R; ++r)
      if (c.failed[r]) c.frozen[r] = 1;
  }
  corner_spectra(c, c.spec.as<double>());
  replica_deltas(c, c.spec.as<double>(), c.specprev.as<double>());
  d2h(c, host_delta, c.delta.as<double>(), c.R);
}

void replica_reset(Context& c, int r, const double* tensors, uint64_t seed) {
  CTM_CHECK(r >= 0 && r < c.R, -1, "replica_reset: no such slot");
  const int N = c.N, NS = c.NS(), s0 = r * N;
  const long cc = (long)c.chi * c.chi, tt = cc * c.Db;
  for (long i = 0; i < (long)N * c.szk; ++i) CTM_CHECK(std::isfinite(tensors[i]), -4, "site tensor has NaN/Inf entries");
  // site tensors, four rotations each (host staging lives until the sync below)
  std::vector<double> ket((size_t)4 * N * c.szk), bra((size_t)4 * N * c.szb, 0.0);
  for (int i = 0; i < N; ++i) {
    std::vector<double> t(tensors + (long)i * c.szk, tensors + (long)(i + 1) * c.szk), rt;
    for (int rot = 0; rot < 4; ++rot) {
      std::copy(t.begin(), t.end(), ket.begin() + ((long)rot * N + i) * c.szk);
      if (c.layers == 2)
        std::copy(t.begin(), t.end(), bra.begin() + ((long)rot * N + i) * c.szb);
      else
        bra[(long)rot * N + i] = 1.0;
      rotate_host(t, rt, c.DK, c.d);
      t.swap(rt);
    }
  }
  for (int rot = 0; rot < 4; ++rot) {
    CTM_HIP(hipMemcpyAsync(c.Aket.as<double>() + ((long)rot * NS + s0) * c.szk, ket.data() + (long)rot * N * c.szk,
                           sizeof(double) * N * c.szk, hipMemcpyHostToDevice, c.st));
    CTM_HIP(hipMemcpyAsync(c.Abra.as<double>() + ((long)rot * NS + s0) * c.szb, bra.data() + (long)rot * N * c.szb,
                           sizeof(double) * N * c.szb, hipMemcpyHostToDevice, c.st));
  }
  // trivial environment: C = [[1]], T[0][0][:] = the ket/bra identity (or ones)
  std::vector<double> hc((size_t)4 * N * cc, 0.0), ht((size_t)4 * N * tt, 0.0);
  for (int k = 0; k < 4 * N; ++k) {
    hc[k * cc] = 1.0;
    for (int b = 0; b < c.Db; ++b)
      ht[k * tt + b] = (c.layers == 2) ? ((b / c.D == b % c.D) ? 1.0 : 0.0) : 1.0;
  }
  CTM_HIP(hipMemcpyAsync(c.C(s0, 0), hc.data(), sizeof(double) * hc.size(), hipMemcpyHostToDevice, c.st));
  CTM_HIP(hipMemcpyAsync(c.Ta(s0, 0), ht.data(), sizeof(double) * ht.size(), hipMemcpyHostToDevice, c.st));
  for (int i = 0; i < N; ++i)
    for (int k = 0; k < 4; ++k) swap_last2(c.st, c.Ta(s0 + i, k), c.Tb(s0 + i, k), c.chi, c.chi, c.Db);
  for (int i = 0; i < N; ++i) {
    c.cdim[s0 + i] = {{{1, 1}, {1, 1}, {1, 1}, {1, 1}}};
    c.tdim[s0 + i] = {{{1, 1}, {1, 1}, {1, 1}, {1, 1}}};
  }
  // reference spectra: every corner [[1]] has the normalised spectrum (1, 0, ..)
  std::vector<double> sp((size_t)4 * N * c.chi, 0.0);
  for (int k = 0; k < 4 * N; ++k) sp[(long)k * c.chi] = 1.0;
  CTM_HIP(hipMemcpyAsync(c.specprev.as<double>() + (long)s0 * 4 * c.chi, sp.data(), sizeof(double) * sp.size(),
                         hipMemcpyHostToDevice, c.st));
  CTM_HIP(hipStreamSynchronize(c.st));
  c.rmoves[r] = 0;
  c.seeds[r] = seed;
  c.frozen[r] = 0;
  c.failed[r] = 0;
}

void do_sweeps_group(Context& c, const int* max_sweeps, const double* tol, int* done, double* delta,
                     int* converged, const std::atomic<bool>* const* cancel) {
  const int R = c.R;
  group_start(c);
  std::vector<double> dl(R, INFINITY);
  for (int r = 0; r < R; ++r) {
    done[r] = 0;
    converged[r] = 0;
    c.frozen[r] = (max_sweeps[r] <= 0) ? 1 : 0;
  }
  for (;;) {
    bool live = false;
    for (int r = 0; r < R; ++r) {
      if (!c.frozen[r] && cancel && cancel[r] && cancel[r]->load()) c.frozen[r] = 1;
      live |= !c.frozen[r];
    }
    if (!live) break;
    std::vector<char> was_live(R);
    for (int r = 0; r < R; ++r) was_live[r] = !c.frozen[r];
    std::vector<double> h(R);
    group_sweep(c, h.data());
    for (int r = 0; r < R; ++r) {
      if (!was_live[r]) continue;
      done[r] += 1;
      dl[r] = h[r];
      if (dl[r] < tol[r]) converged[r] = 1;
      if (converged[r] || done[r] >= max_sweeps[r] || c.failed[r]) c.frozen[r] = 1;
    }
  }
  for (int r = 0; r < R; ++r) {
    delta[r] = dl[r];
    c.frozen[r] = 0;
  }
}

void do_sweeps(Context& c, int max_sweeps, double tol, int* done, double* delta, int* converged,
               const std::atomic<bool>* cancel) {
  CTM_CHECK(c.R == 1, -1, "do_sweeps: one replica");
  int d = 0, conv = 0;
  double dl = INFINITY;
  const std::atomic<bool>* cancels[1] = {cancel};
  do_sweeps_group(c, &max_sweeps, &tol, &d, &dl, &conv, cancel ? cancels : nullptr);
  if (done) *done = d;
  if (delta) *delta = dl;
  if (converged) *converged = conv;
}

}  // namespace ctm
