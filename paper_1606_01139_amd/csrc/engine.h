// Host-side engine of libtransec_gpu: the context, the batched window
// solver, Algorithm 2 and the transmission.  Internal; the C-ABI wraps it.
#pragma once
#include <memory>
#include <new>
#include <string>
#include <utility>
#include <vector>

#include "kernels.h"
#include "transec_gpu.h"

namespace tsg {

struct InvalidArg {
  std::string what;
  explicit InvalidArg(std::string w) : what(std::move(w)) {}
};
struct StateError {
  std::string what;
  explicit StateError(std::string w) : what(std::move(w)) {}
};
struct NotConverged {
  std::string what;
  explicit NotConverged(std::string w) : what(std::move(w)) {}
};
struct OutOfMemory {
  std::string what;
  explicit OutOfMemory(std::string w) : what(std::move(w)) {}
};

// Owning device array.
template <typename T> struct DevArr {
  T* p = nullptr;
  size_t n = 0;
  DevArr() = default;
  DevArr(const DevArr&) = delete;
  DevArr& operator=(const DevArr&) = delete;
  DevArr(DevArr&& o) noexcept : p(o.p), n(o.n) { o.p = nullptr; o.n = 0; }
  DevArr& operator=(DevArr&& o) noexcept {
    if (this != &o) { release(); p = o.p; n = o.n; o.p = nullptr; o.n = 0; }
    return *this;
  }
  ~DevArr() { release(); }
  void alloc(size_t cnt) {
    release();
    if (cnt == 0) return;
    void* q = nullptr;
    if (hipMalloc(&q, cnt * sizeof(T)) != hipSuccess) {
      (void)hipGetLastError();
      throw OutOfMemory("device allocation of " + std::to_string(cnt * sizeof(T)) + " bytes failed");
    }
    p = static_cast<T*>(q);
    n = cnt;
  }
  void ensure(size_t cnt) { if (cnt > n) alloc(cnt); }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    n = 0;
  }
};

struct Partition {
  double shift = 0.0, shift_im = 0.0;
  int nev = 0;
  std::vector<c128> eps;   // ascending real part
  DevArr<c128> U;          // N x n, contiguous columns (ld = N), c-normalised
  tsg_window_stats stats{};
};

struct WindowSpec {
  double shift;
  int nev;
  double shift_im = 0.0;
};

}  // namespace tsg

struct tsg_ctx {
  int nx = 0, ny = 0, nz = 0, R = 6;
  double h = 0.0;
  int64_t N = 0;
  tsg_absorber ab{};
  hipStream_t st = nullptr;
  double coef[7] = {0, 0, 0, 0, 0, 0, 0};  // -c_m / (2h^2)
  double diag0 = 0.0;                      // 3 (-c_0 / (2h^2))
  double normA = 0.0;                      // Gershgorin bound ||A||_G
  double vmin = 0.0, vmax = 0.0, gmax = 0.0;
  std::vector<double> Vh;                  // host copy of V (window planning)
  tsg::DevArr<double> V, gam, gL, gR;      // FP64 operator data (gam, gL, gR per z plane)
  tsg::DevArr<float> Vf, gamf;             // complex64 path
  tsg::SysDesc sys{};                      // this system for the stencil
  tsg::DevArr<tsg::SysDesc> sysd;          // the same, on the device
  std::vector<tsg::Partition> parts;
  // combined set
  bool have_combined = false;
  std::vector<tsg::c128> epsc;
  std::vector<int> ownerc;
  tsg::DevArr<tsg::c128> Uc;
  int nc = 0;
  std::vector<uint8_t> holes;
  // transmission cache
  bool have_grams = false;
  tsg::DevArr<tsg::c128> MR, ML, Wt, epsd;
  std::string err;
};

namespace tsg {

void validate_build(const tsg_grid* g, const double* V, const tsg_absorber* ab);
void build_context(tsg_ctx* c, const tsg_grid* g, const double* V, const tsg_absorber* ab, void* stream);
void apply_operator(tsg_ctx* c, const void* X, void* Y, int ncols, int64_t ld, int dtype);
// Solves the windows together and stores them as new partitions (appended).
// Returns true when every window converged.
bool solve_windows(tsg_ctx* c, const std::vector<WindowSpec>& wins, const tsg_opts& o);
// Windows of several systems in one batched iteration; system s's
// partitions replace those of ctx[s] and are combined.  ok[s] reports
// convergence of every window of system s.
void solve_batch(const std::vector<tsg_ctx*>& ctx, const std::vector<std::vector<WindowSpec>>& wins,
                 const tsg_opts& o, std::vector<bool>& ok);
void combine(tsg_ctx* c, int keep_lowest);
double upper_bound_real(const tsg_ctx* c);
struct FillResult {
  int added = 0, rounds = 0, holes_left = 0;
  bool converged = true;
};
FillResult fill_holes(tsg_ctx* c, double e_min, int n_cap, int max_rounds, const tsg_opts& o);
void plan_windows(tsg_ctx* c, int n_r, int p, int mode, const tsg_opts& o, std::vector<WindowSpec>& out,
                  double* e_range);
void transmission(tsg_ctx* c, const double* E, int nE, double* T);
// Gradient of sum_e w[e] T(E[e]) with respect to V (N values) and
// (amp_L, width_L, amp_R, width_R); returns the COCR iterations used, or
// throws NotConverged.
int transmission_vjp(tsg_ctx* c, const double* E, int nE, const double* w, double* dV, double* dabs);
void dense_eig(void* H, int m, int batch, void* theta, void* Y, int* info, hipStream_t st);
// The same with its workspace in the fixed per-device scratch (noalloc.hip):
// allocates nothing and returns without synchronising.
void dense_eig_noalloc(void* H, int m, int batch, void* theta, void* Y, int* info, hipStream_t st);
int64_t noalloc_scratch_bytes();
// Stencil autotuner (tune.hip).
StencilTuneEntry tune_stencil(tsg_ctx* c, int ncols, int dtype, int reps, int* n_tried);
void write_tuning(const std::string& path);
int load_tuning(const std::string& path);

}  // namespace tsg
