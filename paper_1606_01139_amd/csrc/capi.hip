// extern "C" boundary of libtransec_gpu (declared in include/transec_gpu.h).
// Every entry point converts internal exceptions into a tsg_status and a
// message retrievable with tsg_last_error().
#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "engine.h"

namespace {
thread_local std::string g_last_error;

template <typename F>
tsg_status guarded(tsg_ctx* ctx, F&& f) {
  std::string msg;
  tsg_status s = TSG_OK;
  try {
    s = f();
  } catch (const tsg::InvalidArg& e) {
    s = TSG_EINVAL; msg = e.what;
  } catch (const tsg::StateError& e) {
    s = TSG_ESTATE; msg = e.what;
  } catch (const tsg::NotConverged& e) {
    s = TSG_ENOCONV; msg = e.what;
  } catch (const tsg::OutOfMemory& e) {
    s = TSG_ENOMEM; msg = e.what;
  } catch (const tsg::DeviceError& e) {
    s = TSG_EDEVICE; msg = e.what;
  } catch (const std::bad_alloc&) {
    s = TSG_ENOMEM; msg = "host allocation failed";
  } catch (...) {
    s = TSG_EDEVICE; msg = "unexpected internal error";
  }
  if (s != TSG_OK && !msg.empty()) {
    g_last_error = msg;
    if (ctx) ctx->err = msg;
  }
  return s;
}

// Status of a solve that stored partitions [first, end) of ctx: a dropped
// pair whose u^T u vanished (TSG_EBREAKDOWN) takes precedence over a window
// that did not converge (TSG_ENOCONV).
tsg_status solve_status(tsg_ctx* ctx, size_t first, bool converged) {
  for (size_t j = first; j < ctx->parts.size(); ++j)
    if (ctx->parts[j].stats.cnorm_failures > 0) {
      ctx->err = "a converged pair had u^T u = 0 and could not be c-normalised; it was dropped";
      g_last_error = ctx->err;
      return TSG_EBREAKDOWN;
    }
  if (!converged) {
    ctx->err = "a window did not converge within max_restarts; the converged subset is kept";
    g_last_error = ctx->err;
    return TSG_ENOCONV;
  }
  return TSG_OK;
}

tsg_status fail(tsg_ctx* ctx, tsg_status s, const std::string& msg) {
  g_last_error = msg;
  if (ctx) ctx->err = msg;
  return s;
}

bool device_ok(std::string& why) {
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess || n < 1) {
    (void)hipGetLastError();
    why = "no HIP device available";
    return false;
  }
  int dev = 0;
  hipDeviceProp_t prop;
  if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) {
    why = "cannot query the current HIP device";
    return false;
  }
  if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0) {
    why = std::string("device is ") + prop.gcnArchName + ", this library is built for gfx950";
    return false;
  }
  return true;
}
}  // namespace

extern "C" {

void tsg_default_opts(tsg_opts* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->precision = TSG_FP64;
  o->tol = 1e-8;
  o->block = 2;
  o->basis = 0;
  o->keep = 0;
  o->max_restarts = 2000;
  o->seed = 12345;
  o->keep_lowest = 0;
  o->select = TSG_SELECT_NEAREST;
  o->bulk_tol = 1e-5;
  o->graphs = 1;
  o->groups = 1;
  o->extraction = TSG_EXTRACT_RITZ;
  o->imag_bands = 1;
}

tsg_status tsg_build_operator(const tsg_grid* grid, const double* V, const tsg_absorber* ab, void* hip_stream,
                              tsg_ctx** out) {
  if (!out) return fail(nullptr, TSG_EINVAL, "out is NULL");
  *out = nullptr;
  if (!grid || !V || !ab) return fail(nullptr, TSG_EINVAL, "null argument");
  tsg_status v = guarded(nullptr, [&]() {
    tsg::validate_build(grid, V, ab);
    return TSG_OK;
  });
  if (v != TSG_OK) return v;
  std::string why;
  if (!device_ok(why)) return fail(nullptr, TSG_EDEVICE, why);
  tsg_ctx* c = nullptr;
  try {
    c = new tsg_ctx();
  } catch (...) {
    return fail(nullptr, TSG_ENOMEM, "host allocation failed");
  }
  tsg_status s = guarded(nullptr, [&]() {
    tsg::build_context(c, grid, V, ab, hip_stream);
    return TSG_OK;
  });
  if (s != TSG_OK) {
    delete c;
    return s;
  }
  *out = c;
  return TSG_OK;
}

tsg_status tsg_plan_windows(tsg_ctx* ctx, int32_t n_r, int32_t p, int32_t mode, const tsg_opts* opts,
                            tsg_window* out, double* e_range) {
  if (!ctx || !out) return fail(ctx, TSG_EINVAL, "null argument");
  return guarded(ctx, [&]() {
    tsg_opts o;
    if (opts) o = *opts; else tsg_default_opts(&o);
    std::vector<tsg::WindowSpec> w;
    tsg::plan_windows(ctx, n_r, p, mode, o, w, e_range);
    if (int(w.size()) != p) throw tsg::InvalidArg("planner produced a different number of windows");
    for (int j = 0; j < p; ++j) { out[j].shift = w[j].shift; out[j].nev = w[j].nev; out[j].shift_im = w[j].shift_im; }
    return TSG_OK;
  });
}

tsg_status tsg_solve_partition(tsg_ctx* ctx, tsg_window win, const tsg_opts* opts, int32_t* n_conv) {
  if (!ctx) return fail(ctx, TSG_EINVAL, "ctx is NULL");
  return guarded(ctx, [&]() {
    tsg_opts o;
    if (opts) o = *opts; else tsg_default_opts(&o);
    const size_t first = ctx->parts.size();
    const bool ok = tsg::solve_windows(ctx, {tsg::WindowSpec{win.shift, win.nev, win.shift_im}}, o);
    if (n_conv) *n_conv = ctx->parts.back().stats.n_conv;
    return solve_status(ctx, first, ok);
  });
}

tsg_status tsg_combine(tsg_ctx* ctx, int32_t keep_lowest, int32_t* n_unique, uint8_t* hole_flags) {
  if (!ctx) return fail(ctx, TSG_EINVAL, "ctx is NULL");
  return guarded(ctx, [&]() {
    tsg::combine(ctx, keep_lowest);
    if (n_unique) *n_unique = ctx->nc;
    if (hole_flags)
      for (size_t i = 0; i < ctx->holes.size(); ++i) hole_flags[i] = ctx->holes[i];
    return TSG_OK;
  });
}

tsg_status tsg_solve_all_partitions(tsg_ctx* ctx, const tsg_window* windows, int32_t p, const tsg_opts* opts,
                                    int32_t* n_unique, uint8_t* hole_flags) {
  if (!ctx || !windows) return fail(ctx, TSG_EINVAL, "null argument");
  if (p < 1) return fail(ctx, TSG_EINVAL, "p must be >= 1");
  return guarded(ctx, [&]() {
    tsg_opts o;
    if (opts) o = *opts; else tsg_default_opts(&o);
    std::vector<tsg::WindowSpec> w(p);
    for (int j = 0; j < p; ++j) w[j] = tsg::WindowSpec{windows[j].shift, windows[j].nev, windows[j].shift_im};
    ctx->parts.clear();
    const bool ok = tsg::solve_windows(ctx, w, o);
    tsg::combine(ctx, o.keep_lowest);
    if (n_unique) *n_unique = ctx->nc;
    if (hole_flags)
      for (size_t i = 0; i < ctx->holes.size(); ++i) hole_flags[i] = ctx->holes[i];
    return solve_status(ctx, 0, ok);
  });
}

tsg_status tsg_fill_holes(tsg_ctx* ctx, double e_min, int32_t n_cap, int32_t max_rounds, const tsg_opts* opts,
                          int32_t* n_added, int32_t* rounds, int32_t* n_unique, int32_t* holes_left) {
  if (!ctx) return fail(ctx, TSG_EINVAL, "ctx is NULL");
  return guarded(ctx, [&]() {
    tsg_opts o;
    if (opts) o = *opts; else tsg_default_opts(&o);
    const tsg::FillResult r = tsg::fill_holes(ctx, e_min, n_cap, max_rounds, o);
    if (n_added) *n_added = r.added;
    if (rounds) *rounds = r.rounds;
    if (n_unique) *n_unique = ctx->nc;
    if (holes_left) *holes_left = r.holes_left;
    return solve_status(ctx, 0, r.converged);
  });
}

tsg_status tsg_solve_batch(tsg_ctx* const* ctx, int32_t n_sys, const tsg_window* const* windows, const int32_t* p,
                           const tsg_opts* opts, int32_t* n_unique) {
  if (!ctx || !windows || !p) return fail(nullptr, TSG_EINVAL, "null argument");
  if (n_sys < 1) return fail(nullptr, TSG_EINVAL, "n_sys must be >= 1");
  for (int s = 0; s < n_sys; ++s) {
    if (!ctx[s]) return fail(nullptr, TSG_EINVAL, "null context in batch");
    if (p[s] < 1 || !windows[s]) return fail(ctx[s], TSG_EINVAL, "every system needs p >= 1 windows");
  }
  return guarded(ctx[0], [&]() {
    tsg_opts o;
    if (opts) o = *opts; else tsg_default_opts(&o);
    std::vector<tsg_ctx*> cs(ctx, ctx + n_sys);
    std::vector<std::vector<tsg::WindowSpec>> w(n_sys);
    for (int s = 0; s < n_sys; ++s)
      for (int j = 0; j < p[s]; ++j) w[s].push_back(tsg::WindowSpec{windows[s][j].shift, windows[s][j].nev, windows[s][j].shift_im});
    std::vector<bool> ok;
    tsg::solve_batch(cs, w, o, ok);
    bool all = true;
    for (int s = 0; s < n_sys; ++s) {
      if (n_unique) n_unique[s] = cs[s]->nc;
      all = all && ok[s];
    }
    tsg_status st = TSG_OK;
    for (int s = 0; s < n_sys && st != TSG_EBREAKDOWN; ++s) {
      const tsg_status q = solve_status(cs[s], 0, ok[s]);
      if (q != TSG_OK) {
        st = q;
        ctx[0]->err = cs[s]->err;
      }
    }
    (void)all;
    return st;
  });
}

tsg_status tsg_get_eigenvalues(tsg_ctx* ctx, double* re_im, int32_t cap, int32_t* n) {
  if (!ctx || !n) return fail(ctx, TSG_EINVAL, "null argument");
  if (!ctx->have_combined) return fail(ctx, TSG_ESTATE, "no combined eigenpairs");
  *n = ctx->nc;
  if (cap < ctx->nc) return fail(ctx, TSG_ECAPACITY, "capacity too small");
  if (ctx->nc > 0 && !re_im) return fail(ctx, TSG_EINVAL, "re_im is NULL");
  for (int i = 0; i < ctx->nc; ++i) {
    re_im[2 * i] = ctx->epsc[i].re;
    re_im[2 * i + 1] = ctx->epsc[i].im;
  }
  return TSG_OK;
}

tsg_status tsg_get_eigenvectors(tsg_ctx* ctx, void** dev_ptr, int64_t* ld, int32_t* n) {
  if (!ctx || !dev_ptr || !ld || !n) return fail(ctx, TSG_EINVAL, "null argument");
  if (!ctx->have_combined) return fail(ctx, TSG_ESTATE, "no combined eigenpairs");
  *dev_ptr = ctx->Uc.p;
  *ld = ctx->N;
  *n = ctx->nc;
  return TSG_OK;
}

tsg_status tsg_get_partition(tsg_ctx* ctx, int32_t j, double* re_im, int32_t cap, int32_t* n, void** dev_ptr,
                             int64_t* ld) {
  if (!ctx || !n) return fail(ctx, TSG_EINVAL, "null argument");
  if (j < 0 || j >= int(ctx->parts.size())) return fail(ctx, TSG_EINVAL, "partition index out of range");
  const tsg::Partition& P = ctx->parts[j];
  const int cnt = int(P.eps.size());
  *n = cnt;
  if (re_im) {
    if (cap < cnt) return fail(ctx, TSG_ECAPACITY, "capacity too small");
    for (int i = 0; i < cnt; ++i) { re_im[2 * i] = P.eps[i].re; re_im[2 * i + 1] = P.eps[i].im; }
  }
  if (dev_ptr) *dev_ptr = P.U.p;
  if (ld) *ld = ctx->N;
  return TSG_OK;
}

tsg_status tsg_get_stats(tsg_ctx* ctx, int32_t j, tsg_window_stats* stats) {
  if (!ctx || !stats) return fail(ctx, TSG_EINVAL, "null argument");
  if (j < 0 || j >= int(ctx->parts.size())) return fail(ctx, TSG_EINVAL, "partition index out of range");
  *stats = ctx->parts[j].stats;
  return TSG_OK;
}

tsg_status tsg_transmission(tsg_ctx* ctx, const double* E, int32_t nE, double* T) {
  if (!ctx) return fail(ctx, TSG_EINVAL, "ctx is NULL");
  return guarded(ctx, [&]() {
    tsg::transmission(ctx, E, nE, T);
    return TSG_OK;
  });
}

tsg_status tsg_transmission_vjp(tsg_ctx* ctx, const double* E, int32_t nE, const double* dL_dT, double* dL_dV,
                                double* dL_dabs) {
  if (!ctx) return fail(ctx, TSG_EINVAL, "ctx is NULL");
  return guarded(ctx, [&]() {
    tsg::transmission_vjp(ctx, E, nE, dL_dT, dL_dV, dL_dabs);
    return TSG_OK;
  });
}

tsg_status tsg_apply_operator(tsg_ctx* ctx, const void* X, void* Y, int32_t ncols, int64_t ld, int32_t dtype) {
  if (!ctx) return fail(ctx, TSG_EINVAL, "ctx is NULL");
  return guarded(ctx, [&]() {
    tsg::apply_operator(ctx, X, Y, ncols, ld, dtype);
    return TSG_OK;
  });
}

tsg_status tsg_dense_eig(void* H, int32_t m, int32_t batch, void* theta, void* Y, int32_t* info, void* hip_stream) {
  std::string why;
  if (!device_ok(why)) return fail(nullptr, TSG_EDEVICE, why);
  return guarded(nullptr, [&]() {
    tsg::dense_eig(H, m, batch, theta, Y, info, static_cast<hipStream_t>(hip_stream));
    return TSG_OK;
  });
}

tsg_status tsg_dense_eig_noalloc(void* H, int32_t m, int32_t batch, void* theta, void* Y, int32_t* info,
                                 void* hip_stream) {
  std::string why;
  if (!device_ok(why)) return fail(nullptr, TSG_EDEVICE, why);
  return guarded(nullptr, [&]() {
    tsg::dense_eig_noalloc(H, m, batch, theta, Y, info, static_cast<hipStream_t>(hip_stream));
    return TSG_OK;
  });
}

tsg_status tsg_tune_stencil(tsg_ctx* ctx, int32_t ncols, int32_t dtype, int32_t reps, const char* path,
                            int32_t* geometry, double* best_us) {
  if (!ctx) return fail(ctx, TSG_EINVAL, "ctx is NULL");
  return guarded(ctx, [&]() {
    int tried = 0;
    const tsg::StencilTuneEntry e = tsg::tune_stencil(ctx, ncols, dtype, reps, &tried);
    if (path) tsg::write_tuning(path);
    if (geometry) { geometry[0] = e.g.tx; geometry[1] = e.g.yb; geometry[2] = e.g.zchunk; geometry[3] = e.g.xcd; geometry[4] = e.g.nt; geometry[5] = e.g.cb; geometry[6] = tried; }
    if (best_us) *best_us = e.us;
    return TSG_OK;
  });
}

tsg_status tsg_load_tuning(const char* path, int32_t* n_entries) {
  if (!path) return fail(nullptr, TSG_EINVAL, "path is NULL");
  return guarded(nullptr, [&]() {
    const int n = tsg::load_tuning(path);
    if (n_entries) *n_entries = n;
    return TSG_OK;
  });
}

tsg_status tsg_stencil_geometry(int32_t nx, int32_t ny, int32_t nz, int32_t radius, int32_t ncols, int32_t dtype,
                                int32_t* geometry) {
  if (!geometry) return fail(nullptr, TSG_EINVAL, "geometry is NULL");
  if (nx < 1 || ny < 1 || nz < 1 || radius < 1 || radius > 6 || ncols < 1)
    return fail(nullptr, TSG_EINVAL, "grid, radius (1..6) and ncols must be positive");
  if (dtype != TSG_C128 && dtype != TSG_C64) return fail(nullptr, TSG_EINVAL, "dtype must be TSG_C128 or TSG_C64");
  return guarded(nullptr, [&]() {
    bool tuned = false;
    const tsg::StencilGeom g = tsg::stencil_lookup(nx, ny, nz, ncols, dtype == TSG_C128 ? 16 : 8, radius, &tuned);
    geometry[0] = g.tx;
    geometry[1] = g.yb;
    geometry[2] = std::max(1, std::min(g.zchunk, int(nz)));
    geometry[3] = g.xcd;
    geometry[4] = g.nt;
    geometry[5] = g.cb;
    geometry[6] = tuned ? 1 : 0;
    return TSG_OK;
  });
}

const char* tsg_last_error(const tsg_ctx* ctx) {
  if (ctx && !ctx->err.empty()) return ctx->err.c_str();
  return g_last_error.c_str();
}

void tsg_destroy(tsg_ctx* ctx) { delete ctx; }

}  // extern "C"
