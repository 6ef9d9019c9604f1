// Harmonic Ritz extraction for a window's target shift sigma (the cheaper
// variant of the mixed inversion the paper proposes for interior windows
// that converge slowly, Section 2).
//
// With the explicit Rayleigh quotient H = V^H A V of a Hermitian-orthonormal
// Krylov basis, A V = V H + F E^T holds (F: the part of A times the last
// block outside the basis, E: the last b columns of the identity).  The
// harmonic Ritz pairs (sigma + nu, V y) satisfy
//   W^H (W y - nu V y) = 0,  W = (A - sigma) V,
// i.e. (H - sigma)^H (H - sigma) y + E F^H F E^T y = nu (H - sigma)^H y,
// so they are the eigenpairs of
//   H_h = H + (H - sigma)^{-H} E (F^H F) E^T,
// which differs from H in its last b columns only.  One LU factorisation
// with partial pivoting of (H - sigma)^H per window and b right-hand sides
// give the change; the eigen-decomposition of H_h then runs through the
// ordinary small eigensolver, and the wanted pairs' eigenvalue estimates are
// the Rayleigh quotients y^H H y of the harmonic vectors.
//
// Restart: for H_h y = theta y, A V y - theta V y = (F - V X G) E^T y with
// X = (H - sigma)^{-H} E, G = F^H F, so every harmonic vector's residual lies
// in the span of F~ = F - V X G.  Keeping harmonic vectors and continuing
// from F~ (rather than F) keeps the subspace a Krylov subspace (Morgan's
// harmonic restarted Arnoldi).  With F = P R (P the normalised pending block,
// R^H R = G), F~ R^{-1} = P - V (X G R^{-1}); the kernel returns
// X G R^{-1} (m x b) for that update.
#include "kernels.h"

namespace tsg {
namespace {

constexpr int kHT = 1024;

__device__ inline double hsum(double v, double* red) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  __syncthreads();
  if (lane == 0) red[wv] = v;
  __syncthreads();
  double s = 0.0;
  for (int q = 0; q < kHT / 64; ++q) s += red[q];
  return s;
}

// One workgroup per window.  L (m x m scratch) gets the LU factors of
// (H - sigma)^H with partial pivoting, X (m x b scratch) the solution of
// (H - sigma)^H X = E, and then H[:, m-b+q] += sum_p X[:, p] G[p, q]
// (G = F^H F, b x b).  A zero pivot leaves H unchanged for that window.
__global__ __launch_bounds__(kHT) void harmonic_kernel(c128* Hall, int64_t wsh, int m, int b,
                                                       const c128* __restrict__ sigma, const c128* __restrict__ Gall,
                                                       const c128* __restrict__ Rall, int64_t wsg, c128* Lall,
                                                       int64_t wsl, c128* Xall, int64_t wsx, c128* XGall,
                                                       const int* __restrict__ wmap) {
  const int w = wmap ? wmap[blockIdx.x] : blockIdx.x;
  if (w < 0) return;
  __shared__ double red[kHT / 64];
  __shared__ double bv[kHT / 64];
  __shared__ int bi[kHT / 64];
  __shared__ int piv_s;
  __shared__ int singular;
  c128* H = Hall + int64_t(w) * wsh;
  c128* L = Lall + int64_t(w) * wsl;
  c128* X = Xall + int64_t(w) * wsx;
  c128* XG = XGall + int64_t(w) * wsx;
  const c128* G = Gall + int64_t(w) * wsg;
  const c128* Ri = Rall + int64_t(w) * wsg;
  const c128 sg = conj(sigma[w]);
  const int t = threadIdx.x;
  // L = (H - sigma)^H
  for (int64_t e = t; e < int64_t(m) * m; e += kHT) {
    const int i = int(e / m), j = int(e % m);
    c128 v = conj(H[int64_t(j) * m + i]);
    if (i == j) v = v - sg;
    L[e] = v;
  }
  for (int e = t; e < m * b; e += kHT) {
    const int i = e / b, q = e % b;
    X[e] = c128{i == m - b + q ? 1.0 : 0.0, 0.0};
  }
  if (t == 0) singular = 0;
  __syncthreads();
  for (int k = 0; k < m; ++k) {
    // pivot: largest |L[i][k]|, i >= k
    double best = -1.0;
    int arg = k;
    for (int i = k + t; i < m; i += kHT) {
      const double a = cabs(L[int64_t(i) * m + k]);
      if (a > best) { best = a; arg = i; }
    }
    for (int o = 32; o > 0; o >>= 1) {
      const double ob = __shfl_xor(best, o, 64);
      const int oi = __shfl_xor(arg, o, 64);
      if (ob > best || (ob == best && oi < arg)) { best = ob; arg = oi; }
    }
    if ((t & 63) == 0) { bv[t >> 6] = best; bi[t >> 6] = arg; }
    __syncthreads();
    if (t == 0) {
      double bb = bv[0];
      int ii = bi[0];
      for (int q = 1; q < kHT / 64; ++q)
        if (bv[q] > bb || (bv[q] == bb && bi[q] < ii)) { bb = bv[q]; ii = bi[q]; }
      piv_s = ii;
      if (!(bb > 0.0)) singular = 1;
    }
    __syncthreads();
    if (singular) break;  // H unchanged; XG (zeroed below) leaves the pending block as it is
    const int p = piv_s;
    if (p != k) {
      for (int j = t; j < m; j += kHT) {
        const c128 a = L[int64_t(k) * m + j];
        L[int64_t(k) * m + j] = L[int64_t(p) * m + j];
        L[int64_t(p) * m + j] = a;
      }
      for (int q = t; q < b; q += kHT) {
        const c128 a = X[int64_t(k) * b + q];
        X[int64_t(k) * b + q] = X[int64_t(p) * b + q];
        X[int64_t(p) * b + q] = a;
      }
    }
    __syncthreads();
    const c128 d = L[int64_t(k) * m + k];
    for (int i = k + 1 + t; i < m; i += kHT) L[int64_t(i) * m + k] = cdiv(L[int64_t(i) * m + k], d);
    __syncthreads();
    // trailing update, and the right-hand sides (forward substitution)
    const int rows = m - k - 1, cols = m - k - 1 + b;
    for (int64_t e = t; e < int64_t(rows) * cols; e += kHT) {
      const int i = k + 1 + int(e / cols), c = int(e % cols);
      const c128 l = L[int64_t(i) * m + k];
      if (c < m - k - 1) {
        const int j = k + 1 + c;
        const c128 u = L[int64_t(k) * m + j];
        c128 v = L[int64_t(i) * m + j];
        v.re -= l.re * u.re - l.im * u.im;
        v.im -= l.re * u.im + l.im * u.re;
        L[int64_t(i) * m + j] = v;
      } else {
        const int q = c - (m - k - 1);
        const c128 u = X[int64_t(k) * b + q];
        c128 v = X[int64_t(i) * b + q];
        v.re -= l.re * u.re - l.im * u.im;
        v.im -= l.re * u.im + l.im * u.re;
        X[int64_t(i) * b + q] = v;
      }
    }
    __syncthreads();
  }
  if (singular) {
    for (int e = t; e < m * b; e += kHT) XG[e] = c128{0.0, 0.0};
    return;
  }
  // back substitution U X = Y, one row at a time
  for (int k = m - 1; k >= 0; --k) {
    for (int q = 0; q < b; ++q) {
      c128 s{0.0, 0.0};
      for (int j = k + 1 + t; j < m; j += kHT) fma_acc(s, L[int64_t(k) * m + j], X[int64_t(j) * b + q]);
      const double re = hsum(s.re, red), im = hsum(s.im, red);
      if (t == 0) {
        const c128 v = X[int64_t(k) * b + q] - c128{re, im};
        X[int64_t(k) * b + q] = cdiv(v, L[int64_t(k) * m + k]);
      }
    }
    __syncthreads();
  }
  // H[:, m-b+q] += (X G)[:, q] and XG = X G R^{-1}
  for (int i = t; i < m; i += kHT) {
    c128 xg[kLagMax];
    for (int q = 0; q < b; ++q) {
      c128 acc{0.0, 0.0};
      for (int p2 = 0; p2 < b; ++p2) fma_acc(acc, X[int64_t(i) * b + p2], G[p2 * b + q]);
      xg[q] = acc;
      H[int64_t(i) * m + (m - b + q)] = H[int64_t(i) * m + (m - b + q)] + acc;
    }
    for (int q = 0; q < b; ++q) {
      c128 acc{0.0, 0.0};
      for (int p2 = 0; p2 <= q; ++p2) fma_acc(acc, xg[p2], Ri[p2 * b + q]);
      XG[int64_t(i) * b + q] = acc;
    }
  }
}

// theta[w*nev + i] = y^H H y / y^H y for the columns y = Y[:, off + i]
// (Y row-major m x ld); one wavefront per column.
__global__ __launch_bounds__(256) void rayleigh_kernel(const c128* __restrict__ Hall, int64_t wsh, int m,
                                                       const c128* __restrict__ Yall, int64_t wsy, int ld, int off,
                                                       int nev, c128* theta, int64_t wst,
                                                       const int* __restrict__ wmap) {
  const int w = wmap ? wmap[blockIdx.y] : blockIdx.y;
  if (w < 0) return;
  const int col = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
  if (col >= nev) return;
  const c128* H = Hall + int64_t(w) * wsh;
  const c128* Y = Yall + int64_t(w) * wsy;
  c128 num{0.0, 0.0};
  double den = 0.0;
  for (int i = lane; i < m; i += 64) {
    c128 hy{0.0, 0.0};
    for (int j = 0; j < m; ++j) fma_acc(hy, H[int64_t(i) * m + j], Y[int64_t(j) * ld + off + col]);
    const c128 yi = Y[int64_t(i) * ld + off + col];
    fma_cacc(num, yi, hy);
    den += norm2(yi);
  }
  for (int o = 32; o > 0; o >>= 1) {
    num.re += __shfl_xor(num.re, o, 64);
    num.im += __shfl_xor(num.im, o, 64);
    den += __shfl_xor(den, o, 64);
  }
  if (lane == 0) theta[int64_t(w) * wst + col] = (den > 0.0) ? (1.0 / den) * num : c128{0.0, 0.0};
}

}  // namespace

void harmonic_update(c128* H, int64_t wsh, int m, int b, const c128* sigma, const c128* G, const c128* Rinv,
                     int64_t wsg, c128* L, int64_t wsl, c128* X, int64_t wsx, c128* XG, int nwin, hipStream_t st,
                     const int* wmap) {
  if (nwin <= 0) return;
  if (b > kLagMax) throw DeviceError("harmonic extraction: block size above the supported maximum");
  hipLaunchKernelGGL(harmonic_kernel, dim3(nwin), dim3(kHT), 0, st, H, wsh, m, b, sigma, G, Rinv, wsg, L, wsl, X,
                     wsx, XG, wmap);
}

void rayleigh_quotients(const c128* H, int64_t wsh, int m, const c128* Y, int64_t wsy, int ld, int off, int nev,
                        c128* theta, int64_t wst, int nwin, hipStream_t st, const int* wmap) {
  if (nwin <= 0 || nev <= 0) return;
  hipLaunchKernelGGL(rayleigh_kernel, dim3((nev + 3) / 4, nwin), dim3(256), 0, st, H, wsh, m, Y, wsy, ld, off, nev,
                     theta, wst, wmap);
}

}  // namespace tsg
