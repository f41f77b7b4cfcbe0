// C ABI of libctm (declared in include/ctm.h).
#include <cmath>
#include <complex>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "context.hpp"
#include "kernels.hpp"

struct ctm_ctx {
  ctm::Context c;
  ctm::DevBuf rho;   // small persistent buffer for reduced density matrices
};

// Fixed device array for ctm_expect_2site_noalloc: the transients of the
// bond contraction when the caller cannot allocate.  Each device holds its
// own copy for the life of the process; its address on a device comes from
// hipGetSymbolAddress (the name itself is a host-side stand-in).
constexpr size_t kNoAllocScratchElems = CTM_NOALLOC_SCRATCH_BYTES / sizeof(double);
static __device__ __align__(256) double scratch[kNoAllocScratchElems];

namespace {

constexpr int kMaxDevices = 64;
std::once_flag g_scratch_once[kMaxDevices];
double* g_scratch_ptr[kMaxDevices] = {};
hipError_t g_scratch_err[kMaxDevices] = {};

// Once per device, with that device current: the device address of `scratch`.
void scratch_setup(int dev) {
  if (dev < 0 || dev >= kMaxDevices) return;
  std::call_once(g_scratch_once[dev], [dev] {
    void* p = nullptr;
    g_scratch_err[dev] = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (g_scratch_err[dev] == hipSuccess) g_scratch_ptr[dev] = static_cast<double*>(p);
  });
}

const char* kNullCtx = "null context";
thread_local std::string g_static_err;

template <typename F>
ctm_status guarded(ctm_ctx* ctx, F&& f) {
  try {
    f();
    return CTM_OK;
  } catch (const ctm::Error& e) {
    if (ctx) ctx->c.err = e.what();
    else g_static_err = e.what();
    return (ctm_status)e.status;
  } catch (const std::bad_alloc&) {
    if (ctx) ctx->c.err = "host allocation failed";
    return CTM_ENOMEM;
  } catch (const std::exception& e) {
    if (ctx) ctx->c.err = e.what();
    else g_static_err = e.what();
    return CTM_EDEVICE;
  }
}

bool valid_config(const ctm_config* cfg, std::string& why) {
  if (!cfg) { why = "config is NULL"; return false; }
  if (cfg->Lx < 1 || cfg->Ly < 1 || cfg->Lx * cfg->Ly > 16) { why = "unit cell must have 1..16 sites"; return false; }
  if (cfg->layers != 1 && cfg->layers != 2) { why = "layers must be 1 or 2"; return false; }
  if (cfg->D < 1 || cfg->D > 8) { why = "D must be in 1..8"; return false; }
  if (cfg->layers == 2 && (cfg->d < 1 || cfg->d > 8)) { why = "d must be in 1..8"; return false; }
  if (cfg->layers == 1 && cfg->d != 1) { why = "a classical network (layers = 1) has d = 1"; return false; }
  if (cfg->chi < 1 || cfg->chi > 1024) { why = "chi must be in 1..1024"; return false; }
  if (cfg->prec != CTM_F64 && cfg->prec != CTM_F32 && cfg->prec != CTM_BF16 && cfg->prec != CTM_F16_SPLIT) {
    why = "prec must be CTM_F64, CTM_F32, CTM_BF16 or CTM_F16_SPLIT";
    return false;
  }
  if (cfg->rsvd_power_iters < 0 || cfg->rsvd_power_iters > 8) { why = "rsvd_power_iters must be 0..8"; return false; }
  if (!(cfg->svd_rel_cutoff >= 0.0) || cfg->svd_rel_cutoff >= 1.0) { why = "svd_rel_cutoff must be in [0, 1)"; return false; }
  long Db = (long)cfg->D * (cfg->layers == 2 ? cfg->D : 1);
  long n = cfg->chi * Db;
  if (n * n * (cfg->layers == 2 ? cfg->d : 1) > 2000000000L) { why = "chi * Db too large for 32-bit offsets"; return false; }
  if (cfg->projector_path != CTM_PATH_AUTO && cfg->projector_path != CTM_PATH_HOUSEHOLDER) {
    why = "projector_path must be CTM_PATH_AUTO or CTM_PATH_HOUSEHOLDER";
    return false;
  }
  if (cfg->rsvd_oversample < 0 && n > 8192) { why = "exact SVD mode (rsvd_oversample < 0) needs chi*Db <= 8192"; return false; }
  return true;
}

}  // namespace

ctm::Context& ctm::context_of(ctm_ctx* ctx) { return ctx->c; }

ctm_ctx* ctm::create_group(const ctm_config& cfg, const double* tensors, int replicas, const uint64_t* seeds,
                           ctm_status* st) {
  std::string why;
  if (!valid_config(&cfg, why) || !tensors) {
    *st = CTM_EINVAL;
    return nullptr;
  }
  ctm_ctx* ctx = new (std::nothrow) ctm_ctx();
  if (!ctx) {
    *st = CTM_ENOMEM;
    return nullptr;
  }
  *st = guarded(ctx, [&] {
    ctm::context_init(ctx->c, cfg, tensors, 0, nullptr, replicas, seeds);
    ctx->rho.alloc(sizeof(double) * 4096);
  });
  if (*st != CTM_OK) {
    ctm_free(ctx);
    return nullptr;
  }
  return ctx;
}

extern "C" {

ctm_status ctm_init(const ctm_config* cfg, const double* tensors, int tensors_on_device,
                    const double* boundary, ctm_ctx** out) {
  if (!out) return CTM_EINVAL;
  *out = nullptr;
  std::string why;
  if (!valid_config(cfg, why)) { g_static_err = why; return CTM_EINVAL; }
  if (!tensors) { g_static_err = "tensors is NULL"; return CTM_EINVAL; }
  ctm_ctx* ctx = new (std::nothrow) ctm_ctx();
  if (!ctx) return CTM_ENOMEM;
  ctm_status st = guarded(ctx, [&] {
    ctm::context_init(ctx->c, *cfg, tensors, tensors_on_device, boundary);
    ctx->rho.alloc(sizeof(double) * 4096);
    scratch_setup(ctx->c.device);
  });
  if (st != CTM_OK) {
    g_static_err = ctx->c.err;
    ctm_free(ctx);
    return st;
  }
  *out = ctx;
  return CTM_OK;
}

static int dir_to_rot(int dir) {
  switch (dir) {
    case CTM_LEFT: return 0;
    case CTM_RIGHT: return 2;
    case CTM_UP: return 1;
    case CTM_DOWN: return 3;
    default: return -1;
  }
}

ctm_status ctm_move(ctm_ctx* ctx, ctm_dir dir) {
  if (!ctx) return CTM_EINVAL;
  int rot = dir_to_rot(dir);
  if (rot < 0) { ctx->c.err = "invalid direction"; return CTM_EINVAL; }
  return guarded(ctx, [&] { ctm::do_move(ctx->c, rot); });
}

ctm_status ctm_sweep(ctm_ctx* ctx, int max_sweeps, double tol, int* sweeps_done, double* delta,
                     int* converged) {
  if (!ctx) return CTM_EINVAL;
  if (max_sweeps < 0) { ctx->c.err = "max_sweeps < 0"; return CTM_EINVAL; }
  if (max_sweeps == 0) {
    if (sweeps_done) *sweeps_done = 0;
    if (delta) *delta = 0.0;
    if (converged) *converged = 0;
    return CTM_OK;
  }
  return guarded(ctx, [&] { ctm::do_sweeps(ctx->c, max_sweeps, tol, sweeps_done, delta, converged); });
}

ctm_status ctm_fu_step(ctm_ctx* ctx, const double* H, double tau, int als_iters, int env_sweeps) {
  if (!ctx) return CTM_EINVAL;
  if (!H || als_iters < 0 || env_sweeps < 0) {
    ctx->c.err = "ctm_fu_step: NULL Hamiltonians or negative counts";
    return CTM_EINVAL;
  }
  return guarded(ctx, [&] { ctm::full_update_step(ctx->c, H, tau, als_iters, env_sweeps); });
}

ctm_status ctm_get_tensors(ctm_ctx* ctx, double* tensors) {
  if (!ctx || !tensors) return CTM_EINVAL;
  if (ctx->c.R != 1) { ctx->c.err = "ctm_get_tensors: one solve per context"; return CTM_EINVAL; }
  return guarded(ctx, [&] { ctm::get_site_tensors(ctx->c, tensors); });
}

ctm_status ctm_projectors(ctm_ctx* ctx, ctm_dir dir, int x, int y, double* P, double* Pt, int* k_eff) {
  if (!ctx) return CTM_EINVAL;
  ctm::Context& c = ctx->c;
  int rot = dir_to_rot(dir);
  if (rot < 0) { c.err = "invalid direction"; return CTM_EINVAL; }
  int Lxv = (rot % 2 == 0) ? c.Lx : c.Ly, Lyv = (rot % 2 == 0) ? c.Ly : c.Lx;
  if (x < 0 || x >= Lxv || y < 0 || y >= Lyv) { c.err = "cut outside the unit cell"; return CTM_EINVAL; }
  return guarded(ctx, [&] {
    ctm::cut_projectors_fast(c, rot, x, y);
    const long nc = (long)c.n * c.chi;
    if (Pt) CTM_HIP(hipMemcpyAsync(Pt, c.Pt.p, sizeof(double) * nc, hipMemcpyDeviceToHost, c.st));
    if (P) {
      // P = PT^T: transpose on the device into a panel, then copy
      double* tmp = c.pan[7].as<double>();
      ctm::swap_last2(c.st, c.PT.as<double>(), tmp, 1, c.n, c.chi);
      CTM_HIP(hipMemcpyAsync(P, tmp, sizeof(double) * nc, hipMemcpyDeviceToHost, c.st));
    }
    int ke = c.nact_cut[0];
    if (c.last_cut_svd)   // count the non-zero projector columns
      CTM_HIP(hipMemcpyAsync(&ke, c.keff.p, sizeof(int), hipMemcpyDeviceToHost, c.st));
    CTM_HIP(hipStreamSynchronize(c.st));
    ctm::check_bad(c, "ctm_projectors");
    if (k_eff) *k_eff = ke;
  });
}

ctm_status ctm_enlarged_corner(ctm_ctx* ctx, int corner, int site, double* E) {
  if (!ctx || !E) return CTM_EINVAL;
  ctm::Context& c = ctx->c;
  if (corner < 0 || corner > 3 || site < 0 || site >= c.N) { c.err = "corner / site out of range"; return CTM_EINVAL; }
  return guarded(ctx, [&] {
    ctm::enlarged_corner(c, site, corner, c.G[0].as<double>());
    CTM_HIP(hipMemcpyAsync(E, c.G[0].p, sizeof(double) * c.n * c.n, hipMemcpyDeviceToHost, c.st));
    CTM_HIP(hipStreamSynchronize(c.st));
  });
}

ctm_status ctm_rho_1site(ctm_ctx* ctx, int site, double* rho) {
  if (!ctx) return CTM_EINVAL;
  ctm::Context& c = ctx->c;
  if (site < 0 || site >= c.N || c.layers != 2) { c.err = "site out of range or not an iTPS"; return CTM_EINVAL; }
  return guarded(ctx, [&] { ctm::rho_1site(c, site, ctx->rho.as<double>(), rho); });
}

ctm_status ctm_rho_2site(ctm_ctx* ctx, int site, int dir, double* rho) {
  if (!ctx) return CTM_EINVAL;
  ctm::Context& c = ctx->c;
  if (site < 0 || site >= c.N || (dir != 0 && dir != 1) || c.layers != 2) {
    c.err = "site / dir out of range or not an iTPS";
    return CTM_EINVAL;
  }
  return guarded(ctx, [&] { ctm::rho_2site(c, site, dir, ctx->rho.as<double>(), rho); });
}

ctm_status ctm_expect_1site(ctm_ctx* ctx, int site, const double* op, double* val) {
  if (!ctx || !op || !val) return CTM_EINVAL;
  ctm::Context& c = ctx->c;
  if (site < 0 || site >= c.N || c.layers != 2) { c.err = "site out of range or not an iTPS"; return CTM_EINVAL; }
  return guarded(ctx, [&] { *val = ctm::expect_1site(c, site, op); });
}

ctm_status ctm_expect_2site(ctm_ctx* ctx, int site, int dir, const double* op, double* val) {
  if (!ctx || !op || !val) return CTM_EINVAL;
  ctm::Context& c = ctx->c;
  if (site < 0 || site >= c.N || (dir != 0 && dir != 1) || c.layers != 2) {
    c.err = "site / dir out of range or not an iTPS";
    return CTM_EINVAL;
  }
  return guarded(ctx, [&] { *val = ctm::expect_2site(c, site, dir, op); });
}

ctm_status ctm_expect_2site_noalloc(ctm_ctx* ctx, int site, int dir, const double* op, double* val) {
  if (!ctx || !op || !val) return CTM_EINVAL;
  ctm::Context& c = ctx->c;
  if (site < 0 || site >= c.N || (dir != 0 && dir != 1) || c.layers != 2) {
    c.err = "site / dir out of range or not an iTPS";
    return CTM_EINVAL;
  }
  const int dev = c.device;
  if (dev < 0 || dev >= kMaxDevices || !g_scratch_ptr[dev]) {
    c.err = std::string("no scratch array on this device: ") +
            hipGetErrorString(dev >= 0 && dev < kMaxDevices ? g_scratch_err[dev] : hipErrorInvalidDevice);
    return CTM_EDEVICE;
  }
  const size_t need = ctm::observe_arena_elems(c.chi, c.DK, c.DB, c.d);
  if (need > kNoAllocScratchElems) {
    c.err = "the bond contraction needs " + std::to_string(need * sizeof(double)) +
            " bytes of scratch, more than CTM_NOALLOC_SCRATCH_BYTES";
    return CTM_ETOOBIG;
  }
  ctm::Arena& a = c.arena;
  const auto saved = a.mark();
  a.ext = g_scratch_ptr[dev];
  a.ext_elems = kNoAllocScratchElems;
  const ctm_status st = guarded(ctx, [&] { *val = ctm::expect_2site(c, site, dir, op); });
  a.ext = nullptr;
  a.ext_elems = 0;
  a.release(saved);
  return st;
}

ctm_status ctm_correlation(ctm_ctx* ctx, int site, int dir, const double* opA, const double* opB, int rmax,
                           double* C) {
  if (!ctx || !opA || !opB || !C) return CTM_EINVAL;
  ctm::Context& c = ctx->c;
  if (site < 0 || site >= c.N || (dir != 0 && dir != 1) || rmax < 0 || rmax > 100000 || c.layers != 2) {
    c.err = "site / dir / rmax out of range or not an iTPS";
    return CTM_EINVAL;
  }
  return guarded(ctx, [&] { ctm::correlation(c, site, dir, opA, opB, rmax, C); });
}

ctm_status ctm_transfer_spectrum(ctm_ctx* ctx, int dir, int line, int nev, double* re, double* im, double* e,
                                 double* xi) {
  if (!ctx || !re || !im) return CTM_EINVAL;
  ctm::Context& c = ctx->c;
  if ((dir != 0 && dir != 1) || line < 0 || line >= (dir == 0 ? c.Ly : c.Lx) || nev < 1 || nev > 16) {
    c.err = "dir / line / nev out of range";
    return CTM_EINVAL;
  }
  return guarded(ctx, [&] {
    std::vector<std::complex<double>> lam(nev);
    ctm::transfer_spectrum(c, dir, line, nev, 60, 1e-12, lam.data());
    const int period = (dir == 0) ? c.Lx : c.Ly;
    for (int k = 0; k < nev; ++k) {
      re[k] = lam[k].real();
      im[k] = lam[k].imag();
    }
    const double l0 = std::abs(lam[0]);
    auto ek = [&](int k) {
      const double r = std::abs(lam[k]);
      return (r > 0.0 && l0 > 0.0) ? -std::log(r / l0) / period : INFINITY;
    };
    if (e)
      for (int k = 1; k < nev; ++k) e[k - 1] = ek(k);
    if (xi) *xi = (nev > 1) ? 1.0 / ek(1) : 0.0;
  });
}

ctm_status ctm_xi_extrapolate(int n, const double* e1, const double* e2, double* inv_xi, double* k) {
  if (n < 2 || !e1 || !e2 || !inv_xi || !k) return CTM_EINVAL;
  // least squares for e1 = a + b (e2 - e1): a = 1/xi(inf), b = -k
  double sx = 0, sy = 0, sxx = 0, sxy = 0;
  for (int i = 0; i < n; ++i) {
    const double x = e2[i] - e1[i], y = e1[i];
    if (!std::isfinite(x) || !std::isfinite(y)) return CTM_ENUMERIC;
    sx += x; sy += y; sxx += x * x; sxy += x * y;
  }
  const double den = n * sxx - sx * sx;
  if (!(std::fabs(den) > 0.0)) return CTM_ENUMERIC;
  const double b = (n * sxy - sx * sy) / den;
  *inv_xi = (sy - b * sx) / n;
  *k = -b;
  return CTM_OK;
}

ctm_status ctm_impurity(ctm_ctx* ctx, int site, const double* b, double* val) {
  if (!ctx || !b || !val) return CTM_EINVAL;
  ctm::Context& c = ctx->c;
  if (site < 0 || site >= c.N || c.layers != 1) { c.err = "impurity needs a classical network"; return CTM_EINVAL; }
  return guarded(ctx, [&] { *val = ctm::impurity(c, site, b); });
}

ctm_status ctm_log_kappa(ctm_ctx* ctx, double* ln_kappa) {
  if (!ctx || !ln_kappa) return CTM_EINVAL;
  ctm::Context& c = ctx->c;
  if (c.N != 1) { c.err = "ln kappa needs a 1x1 unit cell"; return CTM_EINVAL; }
  return guarded(ctx, [&] { *ln_kappa = ctm::log_kappa(c); });
}

size_t ctm_env_bytes(const ctm_ctx* ctx) {
  if (!ctx) return 0;
  const ctm::Context& c = ctx->c;
  return sizeof(double) * 4 * ((size_t)c.chi * c.chi + (size_t)c.chi * c.chi * c.Db);
}

ctm_status ctm_get_env(ctm_ctx* ctx, int site, double* buf, size_t bytes, int* dims) {
  if (!ctx || !buf) return CTM_EINVAL;
  ctm::Context& c = ctx->c;
  if (site < 0 || site >= c.N || bytes < ctm_env_bytes(ctx)) { c.err = "site out of range or buffer too small"; return CTM_EINVAL; }
  return guarded(ctx, [&] {
    const long cc = (long)c.chi * c.chi, tt = cc * c.Db;
    CTM_HIP(hipMemcpyAsync(buf, c.C(site, 0), sizeof(double) * 4 * cc, hipMemcpyDeviceToHost, c.st));
    CTM_HIP(hipMemcpyAsync(buf + 4 * cc, c.Ta(site, 0), sizeof(double) * 4 * tt, hipMemcpyDeviceToHost, c.st));
    CTM_HIP(hipStreamSynchronize(c.st));
    if (dims) {
      for (int k = 0; k < 4; ++k) { dims[2 * k] = c.cdim[site][k][0]; dims[2 * k + 1] = c.cdim[site][k][1]; }
      for (int k = 0; k < 4; ++k) { dims[8 + 2 * k] = c.tdim[site][k][0]; dims[8 + 2 * k + 1] = c.tdim[site][k][1]; }
    }
  });
}

ctm_status ctm_set_env(ctm_ctx* ctx, int site, const double* buf, size_t bytes, const int* dims) {
  if (!ctx || !buf) return CTM_EINVAL;
  ctm::Context& c = ctx->c;
  if (site < 0 || site >= c.N || bytes < ctm_env_bytes(ctx)) { c.err = "site out of range or buffer too small"; return CTM_EINVAL; }
  if (dims)
    for (int i = 0; i < 16; ++i)
      if (dims[i] < 1 || dims[i] > c.chi) { c.err = "dims must be in 1..chi"; return CTM_EINVAL; }
  return guarded(ctx, [&] {
    const long cc = (long)c.chi * c.chi, tt = cc * c.Db;
    CTM_HIP(hipMemcpyAsync(c.C(site, 0), buf, sizeof(double) * 4 * cc, hipMemcpyHostToDevice, c.st));
    CTM_HIP(hipMemcpyAsync(c.Ta(site, 0), buf + 4 * cc, sizeof(double) * 4 * tt, hipMemcpyHostToDevice, c.st));
    for (int k = 0; k < 4; ++k) ctm::swap_last2(c.st, c.Ta(site, k), c.Tb(site, k), c.chi, c.chi, c.Db);
    CTM_HIP(hipStreamSynchronize(c.st));
    for (int k = 0; k < 4; ++k) {
      c.cdim[site][k] = {dims ? dims[2 * k] : c.chi, dims ? dims[2 * k + 1] : c.chi};
      c.tdim[site][k] = {dims ? dims[8 + 2 * k] : c.chi, dims ? dims[8 + 2 * k + 1] : c.chi};
    }
  });
}

ctm_status ctm_move_count(const ctm_ctx* ctx, int64_t* moves) {
  if (!ctx || !moves) return CTM_EINVAL;
  *moves = ctx->c.moves;
  return CTM_OK;
}

ctm_status ctm_cut_stats(const ctm_ctx* ctx, int64_t counts[3]) {
  if (!ctx || !counts) return CTM_EINVAL;
  for (int i = 0; i < 3; ++i) counts[i] = ctx->c.cuts[i];
  return CTM_OK;
}

ctm_status ctm_timing_enable(ctm_ctx* ctx, int on) {
  if (!ctx || on < 0 || on > 2) return CTM_EINVAL;
  return guarded(ctx, [&] {
    CTM_HIP(hipStreamSynchronize(ctx->c.st));
    ctx->c.timer.clear();
    // 1: every phase; 2: the sketch GEMMs only
    ctx->c.timer.mask = on == 2 ? (1u << ctm::PhaseTimer::SKETCH) : on ? (1u << ctm::PhaseTimer::N) - 1 : 0u;
  });
}

ctm_status ctm_timing_read(ctm_ctx* ctx, ctm_timing* out) {
  if (!ctx || !out) return CTM_EINVAL;
  return guarded(ctx, [&] {
    ctx->c.timer.resolve();
    for (int i = 0; i < CTM_NPHASE; ++i) {
      out->launches[i] = ctx->c.timer.launches[i];
      out->ms[i] = ctx->c.timer.ms[i];
      out->flops[i] = ctx->c.timer.flops[i];
    }
  });
}

size_t ctm_footprint_bytes(const ctm_config* cfg) {
  std::string why;
  if (!valid_config(cfg, why)) return 0;
  return ctm::context_footprint(*cfg);
}

const char* ctm_last_error(const ctm_ctx* ctx) {
  if (!ctx) return g_static_err.empty() ? kNullCtx : g_static_err.c_str();
  return ctx->c.err.c_str();
}

void ctm_free(ctm_ctx* ctx) {
  if (!ctx) return;
  ctm::Context& c = ctx->c;
  if (c.st) (void)hipStreamSynchronize(c.st);
  ctm::linalg_destroy(c.la);
  c.la = nullptr;
  hipStream_t st = c.st;
  bool own = c.own_stream;
  delete ctx;   // releases every DevBuf
  if (own && st) (void)hipStreamDestroy(st);
}

}  // extern "C"
