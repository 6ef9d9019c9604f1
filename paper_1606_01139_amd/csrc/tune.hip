// Autotuner of the stencil's launch geometry (K1).  The best tile shape is a
// property of the grid shape, the launch width and the element size, and of
// the hardware, so it is measured: every candidate (tile width, points per
// thread in y, z chunk) is launched on the context's grid and timed with HIP
// events on the context's stream; the fastest goes into the in-process table
// that stencil_geometry consults, and optionally into a JSON tuning file.
// The same file read back with tsg_load_tuning restores the table in a later
// process.
#include <algorithm>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>

#include "engine.h"

namespace tsg {
namespace {

std::mutex g_tune_mu;

std::string entry_json(const StencilTuneEntry& x) {
  char buf[256];
  std::snprintf(buf, sizeof(buf),
                "{\"nx\": %d, \"ny\": %d, \"nz\": %d, \"cols\": %d, \"elem\": %d, \"radius\": %d, \"tx\": %d, "
                "\"yb\": %d, \"zchunk\": %d, \"xcd\": %d, \"nt\": %d, \"cb\": %d, \"us\": %.3f}",
                x.nx, x.ny, x.nz, x.cols, x.elem, x.radius, x.g.tx, x.g.yb, x.g.zchunk, x.g.xcd, x.g.nt, x.g.cb, x.us);
  return buf;
}

// Value of "key": <int or number> inside one flat JSON object.
bool field(const std::string& obj, const char* key, double& v) {
  const std::string k = std::string("\"") + key + "\"";
  const size_t p = obj.find(k);
  if (p == std::string::npos) return false;
  const size_t c = obj.find(':', p + k.size());
  if (c == std::string::npos) return false;
  return std::sscanf(obj.c_str() + c + 1, "%lf", &v) == 1;
}

}  // namespace

void write_tuning(const std::string& path) {
  std::lock_guard<std::mutex> lock(g_tune_mu);  // one writer of the file at a time
  FILE* f = std::fopen(path.c_str(), "w");
  if (!f) throw InvalidArg("cannot write the tuning file " + path);
  std::fprintf(f, "{\"stencil\": [\n");
  const std::vector<StencilTuneEntry> e = stencil_tune_table().entries();
  for (size_t i = 0; i < e.size(); ++i)
    std::fprintf(f, "  %s%s\n", entry_json(e[i]).c_str(), i + 1 < e.size() ? "," : "");
  std::fprintf(f, "]}\n");
  std::fclose(f);
}

int load_tuning(const std::string& path) {
  FILE* f = std::fopen(path.c_str(), "r");
  if (!f) throw InvalidArg("cannot read the tuning file " + path);
  std::string text;
  char buf[4096];
  size_t n;
  while ((n = std::fread(buf, 1, sizeof(buf), f)) > 0) text.append(buf, n);
  std::fclose(f);
  const size_t s0 = text.find("\"stencil\"");
  if (s0 == std::string::npos) throw InvalidArg("tuning file has no \"stencil\" list");
  std::vector<StencilTuneEntry> got;
  size_t p = text.find('[', s0);
  while (p != std::string::npos) {
    const size_t a = text.find('{', p), b = text.find('}', a == std::string::npos ? p : a);
    if (a == std::string::npos || b == std::string::npos) break;
    const std::string obj = text.substr(a, b - a + 1);
    double v[10];
    const char* keys[10] = {"nx", "ny", "nz", "cols", "elem", "radius", "tx", "yb", "zchunk", "us"};
    bool ok = true;
    for (int i = 0; i < 10; ++i) ok = ok && field(obj, keys[i], v[i]);
    if (!ok) throw InvalidArg("malformed tuning entry: " + obj);
    double xcd = 0.0, nt = 512.0, cb = 1.0;  // optional keys: launch order, 512 threads, one column
    (void)field(obj, "xcd", xcd);
    (void)field(obj, "nt", nt);
    (void)field(obj, "cb", cb);
    StencilTuneEntry x{int(v[0]), int(v[1]), int(v[2]), int(v[3]), int(v[4]), int(v[5]),
                       StencilGeom{int(v[6]), int(v[7]), int(v[8]), int(xcd), int(nt), int(cb)}, v[9]};
    if (x.cols < 1 || (x.elem != 8 && x.elem != 16) || !stencil_geometry_valid(x.g, x.radius, x.elem))
      throw InvalidArg("invalid tuning entry: " + obj);
    got.push_back(x);
    p = b + 1;
  }
  for (const auto& x : got) stencil_tune_table().put(x);
  return int(got.size());
}

namespace {

template <typename T>
double time_geometry(tsg_ctx* c, const cplx<T>* X, cplx<T>* Y, int ncols, const StencilGeom& gm, int reps,
                     hipEvent_t e0, hipEvent_t e1) {
  StencilArgs<T> a{};
  a.X = X; a.ldx = c->N; a.wsx = 0;
  a.Y = Y; a.ldy = c->N; a.wsy = 0;
  a.ncols = ncols;
  a.radius = c->R;
  a.sys = c->sysd.p;
  a.wsys = nullptr;
  a.wmap = nullptr;
  stencil_apply_geometry(a, c->nx, c->ny, c->nz, gm);
  launch_stencil<T>(a, 1, c->nz, c->st);  // warm-up
  if (hipEventRecord(e0, c->st) != hipSuccess) throw DeviceError("hipEventRecord");
  for (int r = 0; r < reps; ++r) launch_stencil<T>(a, 1, c->nz, c->st);
  if (hipEventRecord(e1, c->st) != hipSuccess) throw DeviceError("hipEventRecord");
  if (hipEventSynchronize(e1) != hipSuccess) throw DeviceError("hipEventSynchronize");
  const hipError_t le = hipGetLastError();
  if (le != hipSuccess) throw DeviceError(std::string("stencil launch: ") + hipGetErrorString(le));
  float ms = 0.f;
  if (hipEventElapsedTime(&ms, e0, e1) != hipSuccess) throw DeviceError("hipEventElapsedTime");
  return 1e3 * double(ms) / reps;
}

template <typename T>
StencilTuneEntry tune_t(tsg_ctx* c, int ncols, int reps, int* n_tried) {
  const int64_t N = c->N;
  DevArr<cplx<T>> X, Y;
  X.alloc(size_t(N) * ncols);
  Y.alloc(size_t(N) * ncols);
  random_block<T>(X.p, N, 0, Rows{N, nullptr}, ncols, 1, 0x7A11u, c->st);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) throw DeviceError("hipEventCreate");
  struct Ev { hipEvent_t a, b; ~Ev() { if (a) (void)hipEventDestroy(a); if (b) (void)hipEventDestroy(b); } } ev{e0, e1};
  const StencilGeom def = stencil_default_geometry(c->nx, c->ny, c->nz, ncols, c->R);
  std::vector<StencilGeom> cand{def};
  for (int nt : {256, 512})
    for (int tx : {16, 32, 64}) {
      if (tx > 2 * std::max(c->nx, 16)) continue;
      for (int yb : {1, 2})
        for (int zc : {16, 24, 32, 48, 64, 96, 128, 192}) {
          if (zc > c->nz && zc != 16) continue;
          for (int xcd : {0, 1})
            for (int cb : {1, 2}) {
              const StencilGeom g{tx, yb, std::min(zc, c->nz), xcd, nt, cb};
              if (stencil_geometry_valid(g, c->R, int(sizeof(cplx<T>)))) cand.push_back(g);
            }
        }
    }
  StencilTuneEntry best{c->nx, c->ny, c->nz, ncols, int(sizeof(cplx<T>)), c->R, def, 1e300};
  for (const StencilGeom& g : cand) {
    const double us = time_geometry<T>(c, X.p, Y.p, ncols, g, reps, e0, e1);
    if (us < best.us) { best.us = us; best.g = g; }
  }
  *n_tried = int(cand.size());
  return best;
}

}  // namespace

StencilTuneEntry tune_stencil(tsg_ctx* c, int ncols, int dtype, int reps, int* n_tried) {
  if (ncols < 1) throw InvalidArg("ncols must be >= 1");
  if (reps < 1) throw InvalidArg("reps must be >= 1");
  StencilTuneEntry e{};
  if (dtype == TSG_C128) e = tune_t<double>(c, ncols, reps, n_tried);
  else if (dtype == TSG_C64) e = tune_t<float>(c, ncols, reps, n_tried);
  else throw InvalidArg("dtype must be TSG_C128 or TSG_C64");
  stencil_tune_table().put(e);
  return e;
}

}  // namespace tsg
