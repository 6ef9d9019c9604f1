// K7 combine helpers (Algorithm 2) and K8 transmission (Section 1).
#include "kernels.h"

namespace tsg {
namespace {

constexpr int kPT = 1024;

__device__ double wg_sum(double v, double* red) {
  const int t = threadIdx.x;
  red[t] = v;
  __syncthreads();
  for (int o = blockDim.x / 2; o > 0; o >>= 1) {
    if (t < o) red[t] += red[t + o];
    __syncthreads();
  }
  const double r = red[0];
  __syncthreads();
  return r;
}

// Algorithm 2's Gram-Schmidt for one eigenpair: v -= v_m (v_m^T v) for each
// partner m in turn (modified Gram-Schmidt, unconjugated product), then
// report ||v||_2 before and after and v^T v.  One workgroup; partners are
// columns of U (c-normalised kept vectors).
__global__ __launch_bounds__(kPT) void project_kernel(c128* v, const c128* U, int64_t ldu, const int* partners,
                                                      int np, int64_t N, double* out) {
  __shared__ double red[kPT];
  const int t = threadIdx.x;
  double b2 = 0.0;
  for (int64_t n = t; n < N; n += kPT) b2 += norm2(v[n]);
  const double before = wg_sum(b2, red);
  for (int q = 0; q < np; ++q) {
    const int m = partners[q];
    double dr = 0.0, di = 0.0;
    for (int64_t n = t; n < N; n += kPT) {
      const c128 a = U[int64_t(m) * ldu + n], b = v[n];
      dr += a.re * b.re - a.im * b.im;
      di += a.re * b.im + a.im * b.re;
    }
    const double cr = wg_sum(dr, red), ci = wg_sum(di, red);
    const c128 c{cr, ci};
    for (int64_t n = t; n < N; n += kPT) v[n] = v[n] - U[int64_t(m) * ldu + n] * c;
    __syncthreads();
  }
  double a2 = 0.0, sr = 0.0, si = 0.0;
  for (int64_t n = t; n < N; n += kPT) {
    const c128 b = v[n];
    a2 += norm2(b);
    sr += b.re * b.re - b.im * b.im;
    si += 2.0 * b.re * b.im;
  }
  const double after = wg_sum(a2, red);
  const double vr = wg_sum(sr, red), vi = wg_sum(si, red);
  if (t == 0) {
    out[0] = sqrt(before);
    out[1] = sqrt(after);
    out[2] = vr;
    out[3] = vi;
  }
}

// dst[:, j] = f_j * src_j  (columns gathered from arbitrary device vectors)
__global__ void gather_kernel(c128* dst, int64_t ldd, const c128* const* srcs, const c128* scale, int64_t N) {
  const int j = blockIdx.y;
  const int64_t row = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (row >= N) return;
  dst[int64_t(j) * ldd + row] = scale[j] * srcs[j][row];
}

// Weighted Grams over the grid: MR = U^T diag(gR) conj U, ML likewise,
// accumulated per row chunk (gamma depends on the z plane only).
constexpr int kWT = 16;
__global__ __launch_bounds__(256) void gamma_gram_partial(const c128* __restrict__ U, int64_t ldu, int64_t N, int n,
                                                          const double* __restrict__ gL, const double* __restrict__ gR,
                                                          int plane, int nchunk, c128* __restrict__ P) {
  __shared__ c128 As[kWT][kWT + 1];
  __shared__ double wl[kWT], wr[kWT];
  const int tiles = (n + kWT - 1) / kWT;
  const int ti = blockIdx.y / tiles, tj = blockIdx.y % tiles;
  const int chunk = blockIdx.x;
  const int64_t rows_per = (N + nchunk - 1) / nchunk;
  const int64_t n0 = chunk * rows_per, n1 = min(N, n0 + rows_per);
  const int tx = threadIdx.x % kWT, ty = threadIdx.x / kWT;
  __shared__ c128 Bs[kWT][kWT + 1];
  c128 accR{0.0, 0.0}, accL{0.0, 0.0};
  for (int64_t nb = n0; nb < n1; nb += kWT) {
    const int64_t row = nb + ty;
    const bool ok = row < n1;
    // As[r][k]: row nb + r of column ti*16 + k (consecutive threads walk rows)
    const int64_t rowc = nb + tx;
    const bool okc = rowc < n1;
    As[tx][ty] = (okc && ti * kWT + ty < n) ? U[int64_t(ti * kWT + ty) * ldu + rowc] : c128{0.0, 0.0};
    Bs[tx][ty] = (okc && tj * kWT + ty < n) ? U[int64_t(tj * kWT + ty) * ldu + rowc] : c128{0.0, 0.0};
    if (tx == 0) {
      wl[ty] = ok ? gL[row / plane] : 0.0;
      wr[ty] = ok ? gR[row / plane] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < kWT; ++q) {
      // entry (k = ti*16+ty, l = tj*16+tx): sum_rows U[row,k] conj(U[row,l]) gamma
      const c128 p = As[q][ty] * conj(Bs[q][tx]);
      accR = accR + wr[q] * p;
      accL = accL + wl[q] * p;
    }
    __syncthreads();
  }
  const int k = ti * kWT + ty, l = tj * kWT + tx;
  if (k < n && l < n) {
    c128* Pw = P + (int64_t(chunk) * n * n + int64_t(k) * n + l) * 2;
    Pw[0] = accR;
    Pw[1] = accL;
  }
}

__global__ void gamma_gram_reduce(const c128* P, int nchunk, int n, c128* MR, c128* ML, c128* W) {
  const int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  const int64_t nn = int64_t(n) * n;
  if (e >= nn) return;
  c128 r{0.0, 0.0}, l{0.0, 0.0};
  for (int c = 0; c < nchunk; ++c) {
    r = r + P[(int64_t(c) * nn + e) * 2];
    l = l + P[(int64_t(c) * nn + e) * 2 + 1];
  }
  MR[e] = r;
  ML[e] = l;
  W[e] = r * l;
}

// One workgroup per energy: T = Re sum_k g_k sum_l W_kl conj(g_l).
__global__ __launch_bounds__(256) void sweep_kernel(const c128* W, int n, const c128* eps, const double* E, double* T) {
  extern __shared__ c128 g[];
  __shared__ double red[256];
  const int e = blockIdx.x;
  const double En = E[e];
  for (int k = threadIdx.x; k < n; k += 256) g[k] = cdiv(c128{1.0, 0.0}, c128{En - eps[k].re, -eps[k].im});
  __syncthreads();
  double acc = 0.0;
  for (int k = threadIdx.x; k < n; k += 256) {
    c128 s{0.0, 0.0};
    for (int l = 0; l < n; ++l) fma_acc(s, W[int64_t(k) * n + l], conj(g[l]));
    const c128 p = g[k] * s;
    acc += p.re;
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) T[e] = red[0];
}

inline int ggram_chunks(int64_t N, int n) {
  const int64_t tiles = int64_t((n + kWT - 1) / kWT) * ((n + kWT - 1) / kWT);
  int64_t want = (4096 + tiles - 1) / tiles;
  const int64_t maxc = (N + 255) / 256;
  if (want > maxc) want = maxc;
  if (want < 1) want = 1;
  return int(want);
}

}  // namespace

int64_t gamma_gram_workspace(int64_t N, int n) { return int64_t(ggram_chunks(N, n)) * n * n * 2; }

template <>
void gamma_grams<double>(const c128* U, int64_t ldu, int64_t N, int n, const double* gL, const double* gR, int plane,
                         c128* MR, c128* ML, c128* W, c128* partials, hipStream_t st) {
  if (n <= 0) return;
  const int nchunk = ggram_chunks(N, n);
  const int tiles = (n + kWT - 1) / kWT;
  hipLaunchKernelGGL(gamma_gram_partial, dim3(nchunk, tiles * tiles), dim3(256), 0, st, U, ldu, N, n, gL, gR, plane,
                     nchunk, partials);
  const int64_t nn = int64_t(n) * n;
  hipLaunchKernelGGL(gamma_gram_reduce, dim3(unsigned((nn + 255) / 256)), dim3(256), 0, st, partials, nchunk, n, MR,
                     ML, W);
}

void transmission_sweep(const c128* W, int n, const c128* eps, const double* E, int nE, double* T, hipStream_t st) {
  if (nE <= 0 || n <= 0) return;
  hipLaunchKernelGGL(sweep_kernel, dim3(nE), dim3(256), size_t(n) * sizeof(c128), st, W, n, eps, E, T);
}

void project_out(c128* v, const c128* U, int64_t ldu, const int* partners, int np, int64_t N, double* out,
                 hipStream_t st) {
  hipLaunchKernelGGL(project_kernel, dim3(1), dim3(kPT), 0, st, v, U, ldu, partners, np, N, out);
}

void gather_columns(c128* dst, int64_t ldd, const c128* const* srcs, const c128* scale, int n, int64_t N,
                    hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(gather_kernel, dim3(unsigned((N + 255) / 256), unsigned(n)), dim3(256), 0, st, dst, ldd, srcs,
                     scale, N);
}

}  // namespace tsg
