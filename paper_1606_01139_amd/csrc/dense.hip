// Batched tall-skinny dense kernels for the window solver:
//   gram        C = X^H Y        (block orthogonalisation, Rayleigh-Ritz)
//   gemm_cols   Y = b Y + a X B  (orthogonalisation update, restart rotation)
//   residuals, c-products, start vectors, copies, small Cholesky.
// Section 1 of Feldman & Zhou: the orthogonalisation of the growing subspace
// and the Rayleigh-Ritz rotations are the O(N n^2) part of the eigensolve.
//
// Layout: every grid vector is contiguous (vector-major).  Column j of the
// block of window w starts at base + w * ws + j * ld; a window's row count
// is rows.of(w), so windows of systems of different size share one launch.
// All reductions over the grid index go through per-chunk partial sums and a
// second fixed-order pass, so results are bitwise reproducible run to run.
#include <algorithm>

#include "kernels.h"

namespace tsg {

namespace {

constexpr int kGT = 64;   // gram tile (rows and columns of C)
constexpr int kGK = 16;   // grid rows of X, Y staged per step

inline int gram_chunks(int64_t N, int r, int s, int nwin) {
  const int64_t tiles = int64_t((r + kGT - 1) / kGT) * ((s + kGT - 1) / kGT) * nwin;
  int64_t want = std::min<int64_t>((4096 + tiles - 1) / tiles, 64);
  int64_t maxc = (N + 511) / 512;
  if (want > maxc) want = maxc;
  if (want < 1) want = 1;
  return int(want);
}

__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// One tile C[i0 : i0 + 64, j0 : j0 + 64] of X^H Y over one chunk of grid
// rows, on the matrix cores.  Complex products are four real ones:
//   Re(conj(x) y) = xr yr + xi yi,   Im(conj(x) y) = xr yi - xi yr,
// each a 16 x 16 x 4 FP64 MFMA (A = X^T, 16 columns by 4 grid rows; B = Y,
// 4 grid rows by 16 columns).  Operand layout of that instruction (measured
// on gfx950 with one-hot inputs): lane l supplies A[l % 16][l / 16] and
// B[l / 16][l % 16] and receives D[l / 16 + 4 v][l % 16] in its v-th
// accumulator (v < 4).  The four
// wavefronts of the workgroup each own a 32 x 32 quarter of the tile
// (2 x 2 blocks of 16 x 16); kGK staged grid rows are 4 k-steps.
typedef double gram_v4d __attribute__((ext_vector_type(4)));

template <typename TX, typename TY>
__global__ __launch_bounds__(256) void gram_mfma_kernel(const cplx<TX>* __restrict__ X, int64_t ldx, int64_t wsx,
                                                        const cplx<TY>* __restrict__ Y, int64_t ldy, int64_t wsy,
                                                        Rows rows, int r, int s, int nchunk,
                                                        c128* __restrict__ P, const int* __restrict__ wmap) {
  // staged rows, real and imaginary parts apart (a lane's 16 neighbours
  // read 16 consecutive doubles)
  __shared__ double Xr[kGK][kGT + 1], Xi[kGK][kGT + 1];
  __shared__ double Yr[kGK][kGT + 1], Yi[kGK][kGT + 1];
  const int wz = blockIdx.z;
  const int w = wmap ? wmap[wz] : wz;
  if (w < 0) return;  // idle slot (whole workgroup)
  const int64_t N = rows.of(w);
  const int tilesJ = (s + kGT - 1) / kGT;
  const int ti = blockIdx.y / tilesJ, tj = blockIdx.y % tilesJ;
  const int chunk = blockIdx.x;
  const int64_t rows_per = ((rows.N + nchunk - 1) / nchunk + kGK - 1) / kGK * kGK;
  const int64_t n0 = chunk * rows_per;
  const int64_t n1 = min(N, n0 + rows_per);
  const int t = threadIdx.x;
  const int lane = t % 64, wave = t / 64;
  const int li = lane % 16, lq = lane / 16;
  const int wi = (wave / 2) * 32, wj = (wave % 2) * 32;  // this wavefront's quarter
  const int i0 = ti * kGT, j0 = tj * kGT;
  X += int64_t(w) * wsx;
  Y += int64_t(w) * wsy;
  gram_v4d cr[2][2], ci[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      cr[a][b] = gram_v4d{0.0, 0.0, 0.0, 0.0};
      ci[a][b] = gram_v4d{0.0, 0.0, 0.0, 0.0};
    }
  for (int64_t nb = n0; nb < n1; nb += kGK) {
    // consecutive threads read consecutive rows of one column
    for (int e = t; e < kGK * kGT; e += 256) {
      const int cc = e / kGK, rr = e % kGK;
      const int64_t n = nb + rr;
      double xr = 0.0, xi = 0.0, yr = 0.0, yi = 0.0;
      if (n < n1) {
        if (i0 + cc < r) { const cplx<TX> v = X[int64_t(i0 + cc) * ldx + n]; xr = double(v.re); xi = double(v.im); }
        if (j0 + cc < s) { const cplx<TY> v = Y[int64_t(j0 + cc) * ldy + n]; yr = double(v.re); yi = double(v.im); }
      }
      Xr[rr][cc] = xr;
      Xi[rr][cc] = xi;
      Yr[rr][cc] = yr;
      Yi[rr][cc] = yi;
    }
    __syncthreads();
#pragma unroll
    for (int ks = 0; ks < kGK / 4; ++ks) {
      const int k = 4 * ks + lq;
      double ar[2], ai[2], br[2], bi[2];
#pragma unroll
      for (int a = 0; a < 2; ++a) {
        ar[a] = Xr[k][wi + 16 * a + li];
        ai[a] = Xi[k][wi + 16 * a + li];
      }
#pragma unroll
      for (int b = 0; b < 2; ++b) {
        br[b] = Yr[k][wj + 16 * b + li];
        bi[b] = Yi[k][wj + 16 * b + li];
      }
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) {
          cr[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(ar[a], br[b], cr[a][b], 0, 0, 0);
          cr[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(ai[a], bi[b], cr[a][b], 0, 0, 0);
          ci[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(ar[a], bi[b], ci[a][b], 0, 0, 0);
          ci[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(-ai[a], br[b], ci[a][b], 0, 0, 0);
        }
    }
    __syncthreads();
  }
  c128* Pw = P + (int64_t(wz) * nchunk + chunk) * int64_t(r) * s;
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int i = i0 + wi + 16 * a + lq + 4 * v, j = j0 + wj + 16 * b + li;
        if (i < r && j < s) Pw[int64_t(i) * s + j] = c128{cr[a][b][v], ci[a][b][v]};
      }
}

__global__ void gram_reduce_kernel(const c128* __restrict__ P, int nchunk, int r, int s, c128* __restrict__ C,
                                   int64_t ldc, int64_t wsc, const int* __restrict__ wmap) {
  const int wz = blockIdx.y;
  const int w = wmap ? wmap[wz] : wz;
  if (w < 0) return;  // idle slot (whole workgroup)
  const int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  const int64_t rs = int64_t(r) * s;
  if (e >= rs) return;
  const c128* Pw = P + int64_t(wz) * nchunk * rs + e;
  c128 acc{0.0, 0.0};
  for (int c = 0; c < nchunk; ++c) acc = acc + Pw[int64_t(c) * rs];
  const int i = int(e / s), j = int(e % s);
  C[int64_t(w) * wsc + int64_t(i) * ldc + j] = acc;
}

// ------------------------------------------------------------- gemm_cols
// Tile of 64 grid rows x 32 output columns per workgroup; each thread owns
// rows tr + 16 q (q < 4) and columns 2 tc, 2 tc + 1, so that a wavefront
// reads and writes runs of 16 consecutive grid rows.
template <typename T>
__global__ __launch_bounds__(256) void gemm_cols_kernel(const cplx<T>* __restrict__ X, int64_t ldx, int64_t wsx,
                                                        const c128* __restrict__ B, int64_t ldb, int64_t wsb,
                                                        cplx<T>* __restrict__ Y, int64_t ldy, int64_t wsy, Rows rows,
                                                        int r, int s, T beta, T alpha,
                                                        const int* __restrict__ wmap) {
  constexpr int TM = 64, TN = 32, KC = 16;
  __shared__ cplx<T> Xs[KC][TM];
  __shared__ cplx<T> Bs[KC][TN];
  const int w = wmap ? wmap[blockIdx.z] : blockIdx.z;
  if (w < 0) return;  // idle slot (whole workgroup)
  const int64_t N = rows.of(w);
  const int64_t r0 = int64_t(blockIdx.x) * TM;
  if (r0 >= N) return;  // whole workgroup, before any barrier
  const int j0 = blockIdx.y * TN;
  const int t = threadIdx.x;
  const int tr = t % 16, tc = t / 16;
  X += int64_t(w) * wsx;
  Y += int64_t(w) * wsy;
  B += int64_t(w) * wsb;
  cplx<T> acc[4][2];
#pragma unroll
  for (int q = 0; q < 4; ++q) acc[q][0] = acc[q][1] = cplx<T>{T(0), T(0)};
  for (int k0 = 0; k0 < r; k0 += KC) {
    for (int e = t; e < TM * KC; e += 256) {
      const int kk = e / TM, rr = e % TM;
      const int64_t n = r0 + rr;
      Xs[kk][rr] = (n < N && k0 + kk < r) ? X[int64_t(k0 + kk) * ldx + n] : cplx<T>{T(0), T(0)};
    }
    for (int e = t; e < KC * TN; e += 256) {
      const int kk = e / TN, jj = e % TN;
      c128 v = (k0 + kk < r && j0 + jj < s) ? B[int64_t(k0 + kk) * ldb + j0 + jj] : c128{0.0, 0.0};
      Bs[kk][jj] = cplx<T>{T(v.re), T(v.im)};
    }
    __syncthreads();
#pragma unroll 4
    for (int kk = 0; kk < KC; ++kk) {
      const cplx<T> b0 = Bs[kk][2 * tc], b1 = Bs[kk][2 * tc + 1];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const cplx<T> x = Xs[kk][tr + 16 * q];
        fma_acc(acc[q][0], x, b0);
        fma_acc(acc[q][1], x, b1);
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int64_t n = r0 + tr + 16 * q;
    if (n >= N) continue;
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      const int j = j0 + 2 * tc + c;
      if (j >= s) continue;
      cplx<T>* y = Y + int64_t(j) * ldy + n;
      cplx<T> v = alpha * acc[q][c];
      if (beta != T(0)) v = v + beta * (*y);
      *y = v;
    }
  }
}

// ------------------------------------------------------------- skinny
// Tall-skinny forms for s <= kSK output columns (the block of new vectors):
// the gram runs one wavefront per column of X; the update streams X once
// with one grid row per thread.
constexpr int kSK = 8;

// Gram for s <= kSK with one wavefront per column of X: the lanes stride
// down the column (contiguous, so every load is a full 1 KiB (c128) run),
// the s columns of Y for the current rows are staged once per workgroup in
// LDS, and each wavefront reduces its s sums at the end of its row chunk.
template <typename TX, typename TY, int S>
__global__ __launch_bounds__(1024) void gram_wave_kernel(const cplx<TX>* __restrict__ X, int64_t ldx, int64_t wsx,
                                                         const cplx<TY>* __restrict__ Y, int64_t ldy, int64_t wsy,
                                                         Rows rows, int r, int s, int nchunk, c128* __restrict__ P,
                                                         const int* __restrict__ wmap) {
  constexpr int KR = 256;
  __shared__ c128 Ys[S][KR];
  const int wz = blockIdx.z;
  const int w = wmap ? wmap[wz] : wz;
  if (w < 0) return;  // idle slot (whole workgroup)
  const int64_t N = rows.of(w);
  const int lane = threadIdx.x % 64, wv = threadIdx.x / 64;
  const int i = blockIdx.y * 16 + wv;
  const int chunk = blockIdx.x;
  const int64_t per = ((rows.N + nchunk - 1) / nchunk + KR - 1) / KR * KR;
  const int64_t n0 = chunk * per, n1 = min(N, n0 + per);
  const bool col_ok = i < r;
  const cplx<TX>* x = X + int64_t(w) * wsx + int64_t(col_ok ? i : 0) * ldx;
  Y += int64_t(w) * wsy;
  double ar[S], ai[S];
#pragma unroll
  for (int q = 0; q < S; ++q) ar[q] = ai[q] = 0.0;
  for (int64_t nb = n0; nb < n1; nb += KR) {
    for (int e = threadIdx.x; e < S * KR; e += 1024) {
      const int q = e / KR, rr = e % KR;
      const int64_t n = nb + rr;
      c128 v{0.0, 0.0};
      if (q < s && n < n1) { const cplx<TY> yv = Y[int64_t(q) * ldy + n]; v = c128{double(yv.re), double(yv.im)}; }
      Ys[q][rr] = v;
    }
    __syncthreads();
    if (col_ok) {
#pragma unroll
      for (int rr = lane; rr < KR; rr += 64) {
        const int64_t n = nb + rr;
        if (n < n1) {
          const cplx<TX> xv = x[n];
          const double xr = double(xv.re), xi = double(xv.im);
#pragma unroll
          for (int q = 0; q < S; ++q) {
            const c128 y = Ys[q][rr];
            // conj(x) * y
            ar[q] = fma(xr, y.re, fma(xi, y.im, ar[q]));
            ai[q] = fma(xr, y.im, fma(-xi, y.re, ai[q]));
          }
        }
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int q = 0; q < S; ++q) {
    ar[q] = wave_sum(ar[q]);
    ai[q] = wave_sum(ai[q]);
  }
  if (col_ok && lane == 0) {
    c128* Pw = P + (int64_t(wz) * nchunk + chunk) * int64_t(r) * s + int64_t(i) * s;
    for (int q = 0; q < s; ++q) Pw[q] = c128{ar[q], ai[q]};
  }
}

template <typename T, int S>
__global__ __launch_bounds__(256) void gemm_skinny_kernel(const cplx<T>* __restrict__ X, int64_t ldx, int64_t wsx,
                                                          const c128* __restrict__ B, int64_t ldb, int64_t wsb,
                                                          cplx<T>* __restrict__ Y, int64_t ldy, int64_t wsy, Rows rows,
                                                          int r, int s, T beta, T alpha,
                                                          const int* __restrict__ wmap) {
  constexpr int KB = 128;
  __shared__ cplx<T> Bs[KB][S];
  const int w = wmap ? wmap[blockIdx.z] : blockIdx.z;
  if (w < 0) return;  // idle slot (whole workgroup)
  const int64_t N = rows.of(w);
  const int64_t n = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (int64_t(blockIdx.x) * 256 >= N) return;  // whole workgroup, before any barrier
  X += int64_t(w) * wsx;
  Y += int64_t(w) * wsy;
  B += int64_t(w) * wsb;
  const bool ok = n < N;
  cplx<T> acc[S];
#pragma unroll
  for (int q = 0; q < S; ++q) acc[q] = cplx<T>{T(0), T(0)};
  for (int k0 = 0; k0 < r; k0 += KB) {
    const int kn = min(KB, r - k0);
    for (int e = threadIdx.x; e < KB * S; e += 256) {
      const int kk = e / S, q = e % S;
      c128 v = (kk < kn && q < s) ? B[int64_t(k0 + kk) * ldb + q] : c128{0.0, 0.0};
      Bs[kk][q] = cplx<T>{T(v.re), T(v.im)};
    }
    __syncthreads();
    if (ok) {
      const cplx<T>* xp = X + int64_t(k0) * ldx + n;
      for (int kk = 0; kk < kn; ++kk) {
        const cplx<T> x = xp[int64_t(kk) * ldx];
#pragma unroll
        for (int q = 0; q < S; ++q) fma_acc(acc[q], x, Bs[kk][q]);
      }
    }
    __syncthreads();
  }
  if (!ok) return;
#pragma unroll
  for (int q = 0; q < S; ++q) {
    if (q >= s) break;
    cplx<T>* y = Y + int64_t(q) * ldy + n;
    cplx<T> v = alpha * acc[q];
    if (beta != T(0)) v = v + beta * (*y);
    *y = v;
  }
}

// ------------------------------------------------------------- column sums
// One workgroup per (row chunk, column, window); per-chunk partials are
// summed in a fixed order by colsum_reduce_kernel.
inline int colsum_chunks(int64_t N, int s, int nwin) {
  const int64_t groups = int64_t(s) * nwin;
  int64_t want = (2048 + groups - 1) / groups;
  int64_t maxc = (N + 2047) / 2048;
  if (want > maxc) want = maxc;
  if (want < 1) want = 1;
  return int(want);
}

template <int NV>
__device__ inline void block_sums(double (&v)[NV], double (*red)[4]) {
  const int lane = threadIdx.x % 64, wv = threadIdx.x / 64;
#pragma unroll
  for (int q = 0; q < NV; ++q) {
    v[q] = wave_sum(v[q]);
    if (lane == 0) red[q][wv] = v[q];
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < NV; ++q) v[q] = red[q][0] + red[q][1] + red[q][2] + red[q][3];
}

template <typename T>
__global__ __launch_bounds__(256) void residual_partial_kernel(const cplx<T>* __restrict__ U, int64_t ldu, int64_t wsu,
                                                               const cplx<T>* __restrict__ AU, int64_t lda, int64_t wsa,
                                                               const c128* __restrict__ theta, int64_t wst, Rows rows,
                                                               int s, int nchunk, double* __restrict__ P,
                                                               const int* __restrict__ wmap) {
  __shared__ double red[2][4];
  const int wz = blockIdx.z;
  const int w = wmap ? wmap[wz] : wz;
  if (w < 0) return;  // idle slot (whole workgroup)
  const int chunk = blockIdx.x, j = blockIdx.y;
  const int64_t N = rows.of(w);
  const int64_t rows_per = (rows.N + nchunk - 1) / nchunk;
  const int64_t n0 = chunk * rows_per, n1 = min(N, n0 + rows_per);
  U += int64_t(w) * wsu + int64_t(j) * ldu;
  AU += int64_t(w) * wsa + int64_t(j) * lda;
  const c128 th = theta[int64_t(w) * wst + j];
  double v[2] = {0.0, 0.0};
  for (int64_t n = n0 + threadIdx.x; n < n1; n += 256) {
    cplx<T> u = U[n], au = AU[n];
    double ur = u.re, ui = u.im;
    double rr = double(au.re) - (th.re * ur - th.im * ui);
    double ri = double(au.im) - (th.re * ui + th.im * ur);
    v[0] += rr * rr + ri * ri;
    v[1] += ur * ur + ui * ui;
  }
  block_sums<2>(v, red);
  if (threadIdx.x == 0) {
    double* Pw = P + ((int64_t(wz) * nchunk + chunk) * s + j) * 2;
    Pw[0] = v[0];
    Pw[1] = v[1];
  }
}

__global__ void colsum_reduce_kernel(const double* __restrict__ P, int nchunk, int s, int width, double* __restrict__ out,
                                     const int* __restrict__ wmap) {
  const int wz = blockIdx.y;
  const int w = wmap ? wmap[wz] : wz;
  if (w < 0) return;  // idle slot (whole workgroup)
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= s * width) return;
  double acc = 0.0;
  for (int c = 0; c < nchunk; ++c) acc += P[(int64_t(wz) * nchunk + c) * s * width + e];
  out[int64_t(w) * s * width + e] = acc;
}

template <typename T>
__global__ __launch_bounds__(256) void cdot_partial_kernel(const cplx<T>* __restrict__ U, int64_t ldu, int64_t wsu,
                                                           const cplx<T>* __restrict__ AU, int64_t lda, int64_t wsa,
                                                           Rows rows, int s, int nchunk, double* __restrict__ P,
                                                           const int* __restrict__ wmap) {
  __shared__ double red[4][4];
  const int wz = blockIdx.z;
  const int w = wmap ? wmap[wz] : wz;
  if (w < 0) return;  // idle slot (whole workgroup)
  const int chunk = blockIdx.x, j = blockIdx.y;
  const int64_t N = rows.of(w);
  const int64_t rows_per = (rows.N + nchunk - 1) / nchunk;
  const int64_t n0 = chunk * rows_per, n1 = min(N, n0 + rows_per);
  U += int64_t(w) * wsu + int64_t(j) * ldu;
  AU += int64_t(w) * wsa + int64_t(j) * lda;
  c128 ua{0.0, 0.0}, uu{0.0, 0.0};
  for (int64_t n = n0 + threadIdx.x; n < n1; n += 256) {
    cplx<T> u = U[n], au = AU[n];
    c128 ud{double(u.re), double(u.im)}, ad{double(au.re), double(au.im)};
    fma_acc(ua, ud, ad);
    fma_acc(uu, ud, ud);
  }
  double v[4] = {ua.re, ua.im, uu.re, uu.im};
  block_sums<4>(v, red);
  if (threadIdx.x == 0) {
    double* Pw = P + ((int64_t(wz) * nchunk + chunk) * s + j) * 4;
    for (int q = 0; q < 4; ++q) Pw[q] = v[q];
  }
}

// F[:, q] = AU[:, sel_q] - theta[sel_q] U[:, sel_q] (explicit residuals of
// selected Ritz pairs); columns with sel_q < 0 are left unchanged.
__device__ inline uint64_t mix64(uint64_t z) {
  z += 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

template <typename T>
__global__ void resblock_kernel(const cplx<T>* __restrict__ U, const cplx<T>* __restrict__ AU, int64_t ld, int64_t ws,
                                const c128* __restrict__ theta, int64_t wst, const int* __restrict__ sel, int b,
                                cplx<T>* __restrict__ F, int64_t ldf, int64_t wsf, Rows rows,
                                const int* __restrict__ wmap) {
  const int w = wmap ? wmap[blockIdx.z] : blockIdx.z;
  if (w < 0) return;  // idle slot (whole workgroup)
  const int q = blockIdx.y;
  const int64_t n = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (n >= rows.of(w)) return;
  const int col = sel[w * b + q];
  if (col < 0) {
    // no pair for this column (a window with fewer wanted pairs): a
    // counter-based random vector keeps the block of full rank
    const uint64_t h = mix64(0xD1B54A32D192ED03ull ^ mix64((uint64_t(w) << 32) ^ uint64_t(q)) ^ mix64(uint64_t(n)));
    const double u = double(h >> 11) * (1.0 / 9007199254740992.0);
    F[int64_t(w) * wsf + int64_t(q) * ldf + n] = cplx<T>{T(2.0 * u - 1.0), T(0)};
    return;
  }
  const c128 th = theta[int64_t(w) * wst + col];
  const int64_t off = int64_t(w) * ws + int64_t(col) * ld + n;
  const cplx<T> u = U[off], au = AU[off];
  const double rr = double(au.re) - (th.re * double(u.re) - th.im * double(u.im));
  const double ri = double(au.im) - (th.re * double(u.im) + th.im * double(u.re));
  F[int64_t(w) * wsf + int64_t(q) * ldf + n] = cplx<T>{T(rr), T(ri)};
}

// ------------------------------------------------------------- misc
template <typename T>
__global__ void random_kernel(cplx<T>* X, int64_t ldx, int64_t wsx, Rows rows, uint64_t seed,
                              const int* __restrict__ wmap) {
  const int w = wmap ? wmap[blockIdx.z] : blockIdx.z;
  if (w < 0) return;  // idle slot (whole workgroup)
  const int j = blockIdx.y;
  const int64_t n = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (n >= rows.of(w)) return;
  uint64_t h = mix64(seed ^ mix64(uint64_t(w) * 0x100000001B3ull + uint64_t(j)) ^ mix64(uint64_t(n) + 0x5851F42Dull));
  double u = double(h >> 11) * (1.0 / 9007199254740992.0);  // [0, 1)
  X[int64_t(w) * wsx + int64_t(j) * ldx + n] = cplx<T>{T(2.0 * u - 1.0), T(0)};
}

// Breakdown of a block step: the new block W (b columns) has lost rank
// against the basis (its Cholesky pivot fell below the floor, flags[w] set),
// i.e. the Krylov space of the window has (numerically) become invariant.
// One workgroup per window replaces W with a counter-based random block,
// made orthogonal to the first J basis columns (and to the earlier columns
// of W) by two classical Gram-Schmidt passes in groups of 8 columns and
// then normalised; Rinv[w] becomes the identity so that the rowmix that
// follows leaves W as it is, and count[w] counts the event.
constexpr int kReseedThreads = 1024;
constexpr int kReseedGroup = 8;

__device__ inline double reseed_sum(double v, double* red) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  __syncthreads();
  if (lane == 0) red[wv] = v;
  __syncthreads();
  double s = 0.0;
  for (int q = 0; q < kReseedThreads / 64; ++q) s += red[q];
  return s;
}

template <typename T>
__global__ __launch_bounds__(kReseedThreads) void reseed_kernel(const cplx<T>* V, int64_t ldv, int64_t wsv, int J,
                                                                cplx<T>* W, int64_t ldw, int64_t wsw, int b, Rows rows,
                                                                const int* __restrict__ flags, int* count, c128* Rinv,
                                                                int64_t wsr, uint64_t seed,
                                                                const int* __restrict__ wmap) {
  const int w = wmap ? wmap[blockIdx.x] : blockIdx.x;
  if (w < 0 || flags[w] == 0) return;
  __shared__ double red[kReseedThreads / 64];
  __shared__ c128 dots[kReseedGroup];
  const int64_t N = rows.of(w);
  const cplx<T>* Vw = V + int64_t(w) * wsv;
  cplx<T>* Ww = W + int64_t(w) * wsw;
  const uint64_t ev = uint64_t(count[w]);
  for (int q = 0; q < b; ++q) {
    cplx<T>* x = Ww + int64_t(q) * ldw;
    for (int64_t n = threadIdx.x; n < N; n += kReseedThreads) {
      const uint64_t h = mix64(seed ^ mix64((uint64_t(w) << 40) ^ (ev << 20) ^ uint64_t(q) ^ 0xA5A5ull) ^
                               mix64(uint64_t(n) + 0x2545F491ull));
      const double u = double(h >> 11) * (1.0 / 9007199254740992.0);
      x[n] = cplx<T>{T(2.0 * u - 1.0), T(0)};
    }
    __syncthreads();
    const int ncol = J + q;
    for (int pass = 0; pass < 2; ++pass) {
      for (int i0 = 0; i0 < ncol; i0 += kReseedGroup) {
        const int g = min(kReseedGroup, ncol - i0);
        c128 acc[kReseedGroup];
#pragma unroll
        for (int t = 0; t < kReseedGroup; ++t) acc[t] = c128{0.0, 0.0};
        for (int64_t n = threadIdx.x; n < N; n += kReseedThreads) {
          const cplx<T> xv = x[n];
          const c128 xd{double(xv.re), double(xv.im)};
#pragma unroll
          for (int t = 0; t < kReseedGroup; ++t) {
            if (t < g) {
              const int i = i0 + t;
              const cplx<T> cv = i < J ? Vw[int64_t(i) * ldv + n] : Ww[int64_t(i - J) * ldw + n];
              fma_cacc(acc[t], c128{double(cv.re), double(cv.im)}, xd);
            }
          }
        }
        for (int t = 0; t < g; ++t) {
          const double re = reseed_sum(acc[t].re, red);
          const double im = reseed_sum(acc[t].im, red);
          if (threadIdx.x == 0) dots[t] = c128{re, im};
        }
        __syncthreads();
        for (int64_t n = threadIdx.x; n < N; n += kReseedThreads) {
          const cplx<T> xv = x[n];
          c128 xd{double(xv.re), double(xv.im)};
          for (int t = 0; t < g; ++t) {
            const int i = i0 + t;
            const cplx<T> cv = i < J ? Vw[int64_t(i) * ldv + n] : Ww[int64_t(i - J) * ldw + n];
            const c128 c{double(cv.re), double(cv.im)};
            const c128 d = dots[t];
            xd.re -= d.re * c.re - d.im * c.im;
            xd.im -= d.re * c.im + d.im * c.re;
          }
          x[n] = cplx<T>{T(xd.re), T(xd.im)};
        }
        __syncthreads();
      }
    }
    double s = 0.0;
    for (int64_t n = threadIdx.x; n < N; n += kReseedThreads) {
      const cplx<T> xv = x[n];
      s += double(xv.re) * double(xv.re) + double(xv.im) * double(xv.im);
    }
    s = reseed_sum(s, red);
    const double inv = s > 0.0 ? 1.0 / sqrt(s) : 0.0;
    for (int64_t n = threadIdx.x; n < N; n += kReseedThreads) {
      const cplx<T> xv = x[n];
      x[n] = cplx<T>{T(inv * double(xv.re)), T(inv * double(xv.im))};
    }
    __syncthreads();
  }
  c128* Ri = Rinv + int64_t(w) * wsr;
  for (int e = threadIdx.x; e < b * b; e += kReseedThreads)
    Ri[e] = c128{(e / b == e % b) ? 1.0 : 0.0, 0.0};
  if (threadIdx.x == 0) count[w] += 1;
}

template <typename TX, typename TY>
__global__ void copy_kernel(const cplx<TX>* X, int64_t ldx, int64_t wsx, cplx<TY>* Y, int64_t ldy, int64_t wsy,
                            Rows rows, const int* __restrict__ wmap) {
  const int w = wmap ? wmap[blockIdx.z] : blockIdx.z;
  if (w < 0) return;  // idle slot (whole workgroup)
  const int j = blockIdx.y;
  const int64_t n = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (n >= rows.of(w)) return;
  cplx<TX> v = X[int64_t(w) * wsx + int64_t(j) * ldx + n];
  Y[int64_t(w) * wsy + int64_t(j) * ldy + n] = cplx<TY>{TY(v.re), TY(v.im)};
}

template <typename T>
__global__ void scale_kernel(cplx<T>* Y, int64_t ldy, int64_t wsy, const c128* scale, int s, Rows rows,
                             const int* __restrict__ wmap) {
  const int w = wmap ? wmap[blockIdx.z] : blockIdx.z;
  if (w < 0) return;  // idle slot (whole workgroup)
  const int j = blockIdx.y;
  const int64_t n = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (n >= rows.of(w)) return;
  c128 f = scale[int64_t(w) * s + j];
  cplx<T>* y = Y + int64_t(w) * wsy + int64_t(j) * ldy + n;
  cplx<T> v = *y;
  *y = cplx<T>{T(f.re * v.re - f.im * v.im), T(f.re * v.im + f.im * v.re)};
}

// One workgroup per window; thread 0 factors G = R^H R (b small) and then
// the workgroup forms R^{-1} column by column.  A pivot that is not
// positive relative to the trace, or not above abs_floor[w] (when given),
// flags a rank-deficient block.
__global__ void cholesky_inv_kernel(const c128* G, int64_t wsg, int b, c128* Rinv, int64_t wsr, int* flags,
                                    const int* __restrict__ wmap, const double* __restrict__ abs_floor) {
  extern __shared__ c128 L[];  // b*b: R (upper), row-major
  const int w = wmap ? wmap[blockIdx.x] : blockIdx.x;
  if (w < 0) return;  // idle slot (whole workgroup)
  const c128* Gw = G + int64_t(w) * wsg;
  c128* Ri = Rinv + int64_t(w) * wsr;
  const int t = threadIdx.x;
  for (int e = t; e < b * b; e += blockDim.x) L[e] = Gw[e];
  __syncthreads();
  __shared__ int bad;
  if (t == 0) {
    bad = 0;
    double tr = 0.0;
    for (int i = 0; i < b; ++i) tr += L[i * b + i].re;
    double floor = 1e-26 * (tr > 0 ? tr : 1.0);
    if (abs_floor) floor = fmax(floor, abs_floor[w]);
    for (int k = 0; k < b; ++k) {
      double d = L[k * b + k].re;
      for (int p = 0; p < k; ++p) d -= norm2(L[p * b + k]);
      if (!(d > floor)) { bad = 1; d = floor > 0 ? floor : 1e-300; }
      d = sqrt(d);
      L[k * b + k] = c128{d, 0.0};
      for (int j = k + 1; j < b; ++j) {
        c128 v = L[k * b + j];
        for (int p = 0; p < k; ++p) v = v - conj(L[p * b + k]) * L[p * b + j];
        L[k * b + j] = (1.0 / d) * v;
      }
      for (int i = k + 1; i < b; ++i) L[i * b + k] = c128{0.0, 0.0};
    }
    flags[w] = bad;
  }
  __syncthreads();
  // R^{-1}: solve R x = e_j for each column j (thread j)
  for (int j = t; j < b; j += blockDim.x) {
    for (int i = b - 1; i >= 0; --i) {
      c128 v = (i == j) ? c128{1.0, 0.0} : c128{0.0, 0.0};
      for (int p = i + 1; p <= j; ++p) v = v - L[i * b + p] * Ri[int64_t(p) * b + j];
      Ri[int64_t(i) * b + j] = (i > j) ? c128{0.0, 0.0} : (1.0 / L[i * b + i].re) * v;
    }
  }
}

// Squared 2-norm of each column: per-chunk partials (one workgroup per
// (chunk, column, window)), summed in a fixed order by colsum_reduce_kernel.
template <typename T>
__global__ __launch_bounds__(256) void colsq_kernel(const cplx<T>* __restrict__ X, int64_t ldx, int64_t wsx, Rows rows,
                                                    int s, int nchunk, double* __restrict__ P,
                                                    const int* __restrict__ wmap) {
  __shared__ double red[1][4];
  const int wz = blockIdx.z;
  const int w = wmap ? wmap[wz] : wz;
  if (w < 0) return;  // idle slot (whole workgroup)
  const int chunk = blockIdx.x, j = blockIdx.y;
  const int64_t N = rows.of(w);
  const int64_t per = (rows.N + nchunk - 1) / nchunk;
  const int64_t n0 = chunk * per, n1 = min(N, n0 + per);
  const cplx<T>* x = X + int64_t(w) * wsx + int64_t(j) * ldx;
  double v[1] = {0.0};
  for (int64_t n = n0 + threadIdx.x; n < n1; n += 256) {
    const cplx<T> a = x[n];
    v[0] += double(a.re) * double(a.re) + double(a.im) * double(a.im);
  }
  block_sums<1>(v, red);
  if (threadIdx.x == 0) P[(int64_t(wz) * nchunk + chunk) * s + j] = v[0];
}

// Second Gram-Schmidt pass only where the first lost more than half of a
// column's squared norm (the criterion of Daniel, Gragg, Kaufman and
// Stewart, eta = 1/sqrt(2)): slot -> window, or -1.
__global__ void dgks_kernel(const double* before, const double* after, int s, int nslot, const int* wmap, int* wmap2) {
  const int slot = blockIdx.x * blockDim.x + threadIdx.x;
  if (slot >= nslot) return;
  const int w = wmap ? wmap[slot] : slot;
  int need = 0;
  if (w >= 0)
    for (int j = 0; j < s; ++j) need |= (after[int64_t(w) * s + j] < 0.5 * before[int64_t(w) * s + j]) ? 1 : 0;
  wmap2[slot] = (w >= 0 && need) ? w : -1;
}

inline dim3 col_grid(int64_t N, int s, int nwin) { return dim3(unsigned((N + 255) / 256), unsigned(s), unsigned(nwin)); }

}  // namespace

// Sized for every active-window count 1..nwin (the chunk count depends on it).
int64_t gram_workspace(int64_t N, int r, int s, int nwin) {
  int64_t best = 0;
  for (int q = 1; q <= nwin; ++q) best = std::max<int64_t>(best, int64_t(gram_chunks(N, r, s, q)) * q);
  return best * r * s;
}

template <typename TX, typename TY>
void gram(const cplx<TX>* X, int64_t ldx, int64_t wsx, const cplx<TY>* Y, int64_t ldy, int64_t wsy, Rows rows,
          int r, int s, c128* C, int64_t ldc, int64_t wsc, int nwin, c128* partials, int64_t cap, hipStream_t st,
          const int* wmap) {
  if (nwin <= 0 || r <= 0 || s <= 0) return;
  const int64_t per = int64_t(nwin) * r * s;
  if (cap < per) throw DeviceError("gram: partial workspace too small");
  int nchunk = int(std::min<int64_t>(gram_chunks(rows.N, r, s, nwin), cap / per));
  if (s <= kSK) {
    // about 2048 workgroups of 16 wavefronts, each wavefront at least 1024 rows
    const int64_t cb = int64_t((r + 15) / 16) * nwin;
    int64_t want = std::max<int64_t>(1, std::min<int64_t>((2048 + cb - 1) / cb, (rows.N + 1023) / 1024));
    nchunk = int(std::min<int64_t>(want, cap / per));
    const dim3 grid(nchunk, (r + 15) / 16, nwin);
    if (s == 1)
      hipLaunchKernelGGL((gram_wave_kernel<TX, TY, 1>), grid, dim3(1024), 0, st, X, ldx, wsx, Y, ldy, wsy, rows, r,
                         s, nchunk, partials, wmap);
    else if (s == 2)
      hipLaunchKernelGGL((gram_wave_kernel<TX, TY, 2>), grid, dim3(1024), 0, st, X, ldx, wsx, Y, ldy, wsy, rows, r,
                         s, nchunk, partials, wmap);
    else if (s <= 4)
      hipLaunchKernelGGL((gram_wave_kernel<TX, TY, 4>), grid, dim3(1024), 0, st, X, ldx, wsx, Y, ldy, wsy, rows, r,
                         s, nchunk, partials, wmap);
    else
      hipLaunchKernelGGL((gram_wave_kernel<TX, TY, kSK>), grid, dim3(1024), 0, st, X, ldx, wsx, Y, ldy, wsy, rows,
                         r, s, nchunk, partials, wmap);
  } else {
    const int tiles = ((r + kGT - 1) / kGT) * ((s + kGT - 1) / kGT);
    hipLaunchKernelGGL((gram_mfma_kernel<TX, TY>), dim3(nchunk, tiles, nwin), dim3(256), 0, st, X, ldx, wsx, Y,
                       ldy, wsy, rows, r, s, nchunk, partials, wmap);
  }
  const int64_t rs = int64_t(r) * s;
  hipLaunchKernelGGL(gram_reduce_kernel, dim3(unsigned((rs + 255) / 256), nwin), dim3(256), 0, st, partials, nchunk,
                     r, s, C, ldc, wsc, wmap);
}

template <typename T>
void gemm_cols(const cplx<T>* X, int64_t ldx, int64_t wsx, const c128* B, int64_t ldb, int64_t wsb, cplx<T>* Y,
               int64_t ldy, int64_t wsy, Rows rows, int r, int s, double beta, int nwin, hipStream_t st,
               const int* wmap, double alpha) {
  if (nwin <= 0 || s <= 0) return;
  if (s <= kSK) {
    const dim3 grid(unsigned((rows.N + 255) / 256), 1, nwin);
    if (s == 1)
      hipLaunchKernelGGL((gemm_skinny_kernel<T, 1>), grid, dim3(256), 0, st, X, ldx, wsx, B, ldb, wsb, Y, ldy, wsy,
                         rows, r, s, T(beta), T(alpha), wmap);
    else if (s == 2)
      hipLaunchKernelGGL((gemm_skinny_kernel<T, 2>), grid, dim3(256), 0, st, X, ldx, wsx, B, ldb, wsb, Y, ldy, wsy,
                         rows, r, s, T(beta), T(alpha), wmap);
    else if (s <= 4)
      hipLaunchKernelGGL((gemm_skinny_kernel<T, 4>), grid, dim3(256), 0, st, X, ldx, wsx, B, ldb, wsb, Y, ldy, wsy,
                         rows, r, s, T(beta), T(alpha), wmap);
    else
      hipLaunchKernelGGL((gemm_skinny_kernel<T, kSK>), grid, dim3(256), 0, st, X, ldx, wsx, B, ldb, wsb, Y, ldy,
                         wsy, rows, r, s, T(beta), T(alpha), wmap);
    return;
  }
  hipLaunchKernelGGL((gemm_cols_kernel<T>), dim3(unsigned((rows.N + 63) / 64), unsigned((s + 31) / 32), nwin),
                     dim3(256), 0, st, X, ldx, wsx, B, ldb, wsb, Y, ldy, wsy, rows, r, s, T(beta), T(alpha), wmap);
}

template <typename T>
void residual_block(const cplx<T>* U, const cplx<T>* AU, int64_t ld, int64_t ws, const c128* theta, int64_t wst,
                    const int* sel, int b, cplx<T>* F, int64_t ldf, int64_t wsf, Rows rows, int nwin, hipStream_t st,
                    const int* wmap) {
  if (nwin <= 0 || b <= 0) return;
  hipLaunchKernelGGL((resblock_kernel<T>), col_grid(rows.N, b, nwin), dim3(256), 0, st, U, AU, ld, ws, theta, wst,
                     sel, b, F, ldf, wsf, rows, wmap);
}
template void residual_block<double>(const c128*, const c128*, int64_t, int64_t, const c128*, int64_t, const int*,
                                     int, c128*, int64_t, int64_t, Rows, int, hipStream_t, const int*);
template void residual_block<float>(const c64*, const c64*, int64_t, int64_t, const c128*, int64_t, const int*, int,
                                    c64*, int64_t, int64_t, Rows, int, hipStream_t, const int*);

int64_t residual_workspace(int64_t N, int s, int nwin) {
  int64_t best = 0;
  for (int q = 1; q <= nwin; ++q) best = std::max<int64_t>(best, int64_t(colsum_chunks(N, s, q)) * q);
  return best * s * 4;
}

template <typename T>
void residual_norms(const cplx<T>* U, int64_t ldu, int64_t wsu, const cplx<T>* AU, int64_t lda, int64_t wsa,
                    const c128* theta, int64_t wst, Rows rows, int s, int nwin, double* out, double* partials,
                    int64_t cap, hipStream_t st, const int* wmap) {
  if (nwin <= 0 || s <= 0) return;
  const int64_t per = int64_t(nwin) * s * 2;
  if (cap < per) throw DeviceError("residual_norms: partial workspace too small");
  const int nchunk = int(std::min<int64_t>(colsum_chunks(rows.N, s, nwin), cap / per));
  hipLaunchKernelGGL((residual_partial_kernel<T>), dim3(nchunk, s, nwin), dim3(256), 0, st, U, ldu, wsu, AU, lda,
                     wsa, theta, wst, rows, s, nchunk, partials, wmap);
  hipLaunchKernelGGL(colsum_reduce_kernel, dim3((2 * s + 255) / 256, nwin), dim3(256), 0, st, partials, nchunk, s, 2,
                     out, wmap);
}

template <typename T>
void cdots(const cplx<T>* U, int64_t ldu, int64_t wsu, const cplx<T>* AU, int64_t lda, int64_t wsa, Rows rows, int s,
           int nwin, c128* out, double* partials, int64_t cap, hipStream_t st, const int* wmap) {
  if (nwin <= 0 || s <= 0) return;
  const int64_t per = int64_t(nwin) * s * 4;
  if (cap < per) throw DeviceError("cdots: partial workspace too small");
  const int nchunk = int(std::min<int64_t>(colsum_chunks(rows.N, s, nwin), cap / per));
  hipLaunchKernelGGL((cdot_partial_kernel<T>), dim3(nchunk, s, nwin), dim3(256), 0, st, U, ldu, wsu, AU, lda, wsa,
                     rows, s, nchunk, partials, wmap);
  hipLaunchKernelGGL(colsum_reduce_kernel, dim3((4 * s + 255) / 256, nwin), dim3(256), 0, st, partials, nchunk, s, 4,
                     reinterpret_cast<double*>(out), wmap);
}

template <typename T>
void random_block(cplx<T>* X, int64_t ldx, int64_t wsx, Rows rows, int s, int nwin, uint64_t seed, hipStream_t st,
                  const int* wmap) {
  if (nwin <= 0 || s <= 0) return;
  hipLaunchKernelGGL((random_kernel<T>), col_grid(rows.N, s, nwin), dim3(256), 0, st, X, ldx, wsx, rows, seed, wmap);
}

template <typename TX, typename TY>
void copy_block(const cplx<TX>* X, int64_t ldx, int64_t wsx, cplx<TY>* Y, int64_t ldy, int64_t wsy, Rows rows, int s,
                int nwin, hipStream_t st, const int* wmap) {
  if (nwin <= 0 || s <= 0) return;
  hipLaunchKernelGGL((copy_kernel<TX, TY>), col_grid(rows.N, s, nwin), dim3(256), 0, st, X, ldx, wsx, Y, ldy, wsy,
                     rows, wmap);
}

template <typename T>
void scale_cols(cplx<T>* Y, int64_t ldy, int64_t wsy, const c128* scale, Rows rows, int s, int nwin, hipStream_t st,
                const int* wmap) {
  if (nwin <= 0 || s <= 0) return;
  hipLaunchKernelGGL((scale_kernel<T>), col_grid(rows.N, s, nwin), dim3(256), 0, st, Y, ldy, wsy, scale, s, rows,
                     wmap);
}

template <typename T>
void col_sqnorms(const cplx<T>* X, int64_t ldx, int64_t wsx, Rows rows, int s, int nwin, double* out, double* partials,
                 int64_t cap, hipStream_t st, const int* wmap) {
  if (nwin <= 0 || s <= 0) return;
  const int64_t per = int64_t(nwin) * s;
  if (cap < per) throw DeviceError("col_sqnorms: partial workspace too small");
  const int nchunk = int(std::min<int64_t>(colsum_chunks(rows.N, s, nwin), cap / per));
  hipLaunchKernelGGL((colsq_kernel<T>), dim3(nchunk, s, nwin), dim3(256), 0, st, X, ldx, wsx, rows, s, nchunk,
                     partials, wmap);
  hipLaunchKernelGGL(colsum_reduce_kernel, dim3((s + 255) / 256, nwin), dim3(256), 0, st, partials, nchunk, s, 1, out,
                     wmap);
}
template void col_sqnorms<double>(const c128*, int64_t, int64_t, Rows, int, int, double*, double*, int64_t,
                                  hipStream_t, const int*);
template void col_sqnorms<float>(const c64*, int64_t, int64_t, Rows, int, int, double*, double*, int64_t, hipStream_t,
                                 const int*);

void dgks_select(const double* before, const double* after, int s, int nslot, const int* wmap, int* wmap2,
                 hipStream_t st) {
  if (nslot <= 0) return;
  hipLaunchKernelGGL(dgks_kernel, dim3((nslot + 63) / 64), dim3(64), 0, st, before, after, s, nslot, wmap, wmap2);
}

// Lagged second Gram-Schmidt pass (one workgroup per window).  G is the
// (j + b) x 2b product [V_j P]^H [P W] of a block step: S = V_j^H P (rows
// 0..j-1, columns 0..b-1), C = V_j^H W (rows 0..j-1, columns b..2b-1),
// P^H P and P^H W (rows j..j+b-1).  After [P W] -= V_j [S C], the pending
// block P' = P - V_j S has Gram P'^H P' = P^H P - S^H S = R^H R and
// P'^H W' = P^H W - S^H C; M (2b x 2b) maps [P' W'] to
// [P' R^-1, W' - P' R^-1 D] with D = R^-H (P^H W - S^H C), i.e. the final
// block and W' made orthogonal to it.
constexpr int kLagThreads = 64 * 2 * kLagMax * kLagMax / 4;  // 8 wavefronts

__global__ __launch_bounds__(kLagThreads) void lagfix_kernel(const c128* G, int64_t wsg, int j, int b, c128* M,
                                                             int64_t wsm, int* flags, const int* __restrict__ wmap) {
  __shared__ c128 A[kLagMax * kLagMax], E[kLagMax * kLagMax], R[kLagMax * kLagMax], Ri[kLagMax * kLagMax];
  const int w = wmap ? wmap[blockIdx.x] : blockIdx.x;
  if (w < 0) return;  // idle slot (whole workgroup)
  const c128* Gw = G + int64_t(w) * wsg;
  c128* Mw = M + int64_t(w) * wsm;
  const int t = threadIdx.x, ld = 2 * b, lane = t & 63;
  // A = P^H P - S^H S and E = P^H W - S^H C: one wavefront per entry, the
  // sum over the basis rows split over its lanes
  for (int e = t >> 6; e < 2 * b * b; e += kLagThreads / 64) {
    const int which = e / (b * b), pq = e % (b * b), p = pq / b, q = pq % b;
    const int col = which ? b + q : q;
    c128 v{0.0, 0.0};
    for (int i = lane; i < j; i += 64) fma_cacc(v, Gw[int64_t(i) * ld + p], Gw[int64_t(i) * ld + col]);
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      v.re += __shfl_xor(v.re, o, 64);
      v.im += __shfl_xor(v.im, o, 64);
    }
    if (lane == 0) (which ? E : A)[p * b + q] = Gw[int64_t(j + p) * ld + col] - v;
  }
  __syncthreads();
  if (t == 0) {
    // Cholesky A = R^H R (R upper), then R^-1
    int bad = 0;
    double tr = 0.0;
    for (int i = 0; i < b; ++i) tr += A[i * b + i].re;
    const double floor = 1e-26 * (tr > 0 ? tr : 1.0);
    for (int k = 0; k < b; ++k) {
      double d = A[k * b + k].re;
      for (int p = 0; p < k; ++p) d -= norm2(R[p * b + k]);
      if (!(d > floor)) { bad = 1; d = floor > 0 ? floor : 1e-300; }
      d = sqrt(d);
      R[k * b + k] = c128{d, 0.0};
      for (int q = k + 1; q < b; ++q) {
        c128 v = A[k * b + q];
        for (int p = 0; p < k; ++p) v = v - conj(R[p * b + k]) * R[p * b + q];
        R[k * b + q] = (1.0 / d) * v;
      }
      for (int i = k + 1; i < b; ++i) R[i * b + k] = c128{0.0, 0.0};
    }
    for (int q = 0; q < b; ++q)
      for (int i = b - 1; i >= 0; --i) {
        c128 v = (i == q) ? c128{1.0, 0.0} : c128{0.0, 0.0};
        for (int p = i + 1; p <= q; ++p) v = v - R[i * b + p] * Ri[p * b + q];
        Ri[i * b + q] = (i > q) ? c128{0.0, 0.0} : (1.0 / R[i * b + i].re) * v;
      }
    // D = R^-H E (lower-triangular solve R^H D = E), kept in A
    for (int q = 0; q < b; ++q)
      for (int i = 0; i < b; ++i) {
        c128 v = E[i * b + q];
        for (int p = 0; p < i; ++p) v = v - conj(R[p * b + i]) * A[p * b + q];
        A[i * b + q] = (1.0 / R[i * b + i].re) * v;
      }
    // M = [[R^-1, -R^-1 D], [0, I]]
    for (int p = 0; p < b; ++p)
      for (int q = 0; q < b; ++q) {
        c128 v{0.0, 0.0};
        for (int i = 0; i < b; ++i) v = v + Ri[p * b + i] * A[i * b + q];
        Mw[p * ld + q] = Ri[p * b + q];
        Mw[p * ld + b + q] = c128{-v.re, -v.im};
        Mw[(b + p) * ld + q] = c128{0.0, 0.0};
        Mw[(b + p) * ld + b + q] = c128{p == q ? 1.0 : 0.0, 0.0};
      }
    flags[w] = bad;
  }
}

// Y[w] (N x s, s <= kLagMax * 2 contiguous columns) <- Y[w] M[w] (s x s,
// row-major), in place: each thread owns one row.
template <typename T>
__global__ __launch_bounds__(256) void rowmix_kernel(cplx<T>* Y, int64_t ldy, int64_t wsy, const c128* M, int64_t wsm,
                                                     Rows rows, int s, const int* __restrict__ wmap) {
  const int w = wmap ? wmap[blockIdx.z] : blockIdx.z;
  if (w < 0) return;  // idle slot (whole workgroup)
  const int64_t n = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (n >= rows.of(w)) return;
  cplx<T>* y = Y + int64_t(w) * wsy + n;
  const c128* Mw = M + int64_t(w) * wsm;
  c128 x[2 * kLagMax];
  for (int p = 0; p < s; ++p) {
    const cplx<T> v = y[int64_t(p) * ldy];
    x[p] = c128{double(v.re), double(v.im)};
  }
  for (int q = 0; q < s; ++q) {
    c128 acc{0.0, 0.0};
    for (int p = 0; p < s; ++p) fma_acc(acc, x[p], Mw[p * s + q]);
    y[int64_t(q) * ldy] = cplx<T>{T(acc.re), T(acc.im)};
  }
}

void lagfix(const c128* G, int64_t wsg, int j, int b, c128* M, int64_t wsm, int* flags, int nwin, hipStream_t st,
            const int* wmap) {
  if (nwin <= 0) return;
  if (b > kLagMax) throw DeviceError("block size too large for the lagged Gram-Schmidt pass");
  hipLaunchKernelGGL(lagfix_kernel, dim3(nwin), dim3(kLagThreads), 0, st, G, wsg, j, b, M, wsm, flags, wmap);
}

template <typename T>
void rowmix(cplx<T>* Y, int64_t ldy, int64_t wsy, const c128* M, int64_t wsm, Rows rows, int s, int nwin,
            hipStream_t st, const int* wmap) {
  if (nwin <= 0 || s <= 0) return;
  if (s > 2 * kLagMax) throw DeviceError("rowmix: too many columns");
  hipLaunchKernelGGL((rowmix_kernel<T>), dim3(unsigned((rows.N + 255) / 256), 1, nwin), dim3(256), 0, st, Y, ldy, wsy,
                     M, wsm, rows, s, wmap);
}
template void rowmix<double>(cplx<double>*, int64_t, int64_t, const c128*, int64_t, Rows, int, int, hipStream_t,
                             const int*);
template void rowmix<float>(cplx<float>*, int64_t, int64_t, const c128*, int64_t, Rows, int, int, hipStream_t,
                            const int*);

void cholesky_inv(const c128* G, int64_t wsg, int b, c128* Rinv, int64_t wsr, int* flags, int nwin, hipStream_t st,
                  const int* wmap, const double* abs_floor) {
  if (nwin <= 0) return;
  hipLaunchKernelGGL(cholesky_inv_kernel, dim3(nwin), dim3(64), size_t(b) * b * sizeof(c128), st, G, wsg, b, Rinv,
                     wsr, flags, wmap, abs_floor);
}

template <typename T>
void reseed_block(const cplx<T>* V, int64_t ldv, int64_t wsv, int J, cplx<T>* W, int64_t ldw, int64_t wsw, int b,
                  Rows rows, const int* flags, int* count, c128* Rinv, int64_t wsr, uint64_t seed, int nwin,
                  hipStream_t st, const int* wmap) {
  if (nwin <= 0 || b <= 0) return;
  hipLaunchKernelGGL((reseed_kernel<T>), dim3(nwin), dim3(kReseedThreads), 0, st, V, ldv, wsv, J, W, ldw, wsw, b,
                     rows, flags, count, Rinv, wsr, seed, wmap);
}
template void reseed_block<double>(const cplx<double>*, int64_t, int64_t, int, cplx<double>*, int64_t, int64_t, int,
                                   Rows, const int*, int*, c128*, int64_t, uint64_t, int, hipStream_t, const int*);
template void reseed_block<float>(const cplx<float>*, int64_t, int64_t, int, cplx<float>*, int64_t, int64_t, int,
                                  Rows, const int*, int*, c128*, int64_t, uint64_t, int, hipStream_t, const int*);

#define TSG_INST_T(T)                                                                                              \
  template void gemm_cols<T>(const cplx<T>*, int64_t, int64_t, const c128*, int64_t, int64_t, cplx<T>*, int64_t,  \
                             int64_t, Rows, int, int, double, int, hipStream_t, const int*, double);               \
  template void residual_norms<T>(const cplx<T>*, int64_t, int64_t, const cplx<T>*, int64_t, int64_t, const c128*, \
                                  int64_t, Rows, int, int, double*, double*, int64_t, hipStream_t, const int*);    \
  template void cdots<T>(const cplx<T>*, int64_t, int64_t, const cplx<T>*, int64_t, int64_t, Rows, int, int,       \
                         c128*, double*, int64_t, hipStream_t, const int*);                                         \
  template void random_block<T>(cplx<T>*, int64_t, int64_t, Rows, int, int, uint64_t, hipStream_t, const int*);   \
  template void scale_cols<T>(cplx<T>*, int64_t, int64_t, const c128*, Rows, int, int, hipStream_t, const int*);
TSG_INST_T(double)
TSG_INST_T(float)

#define TSG_INST_2(TX, TY)                                                                                           \
  template void gram<TX, TY>(const cplx<TX>*, int64_t, int64_t, const cplx<TY>*, int64_t, int64_t, Rows, int, int, \
                             c128*, int64_t, int64_t, int, c128*, int64_t, hipStream_t, const int*);                 \
  template void copy_block<TX, TY>(const cplx<TX>*, int64_t, int64_t, cplx<TY>*, int64_t, int64_t, Rows, int, int, \
                                   hipStream_t, const int*);
TSG_INST_2(double, double)
TSG_INST_2(float, float)
TSG_INST_2(float, double)
TSG_INST_2(double, float)

}  // namespace tsg
