// K4: eigenpairs of the small Rayleigh-Ritz matrix H (m x m, general complex,
// FP64), one workgroup per window.
//
// The paper's solver (ARPACK, Section 2.1) extracts Ritz pairs from the
// projected matrix with a dense QR algorithm; this is the same textbook route
// (Golub & Van Loan, Matrix Computations, Ch. 7): Householder reduction to
// upper Hessenberg form, the implicit single-shift complex QR iteration with
// Wilkinson shifts and deflation (accumulating the Schur vectors), eigenvectors
// of the triangular factor by back substitution, and back-transformation.
//
// Then select_restart orders the Ritz values by |theta - sigma| (the 'SM'
// selection on the shifted operator, Eq. (3) and Section 2.1) and builds the
// thick-restart basis.
#include "kernels.h"

namespace tsg {
namespace {

constexpr int kEigThreads = 512;
constexpr int kSB = 8;  // column block of the restart-basis orthonormalisation
constexpr int kSelThreads = 512;  // threads of select_restart_kernel (a power of two)
// Bases from this size on take the Hessenberg reduction over several
// workgroups per matrix (row slabs of about kSlabRows rows, at most
// kMaxSlabs).
constexpr int kSlabMinBasis = 192;
#ifndef TSG_HESS_SLAB_ROWS
#define TSG_HESS_SLAB_ROWS 32
#endif
#ifndef TSG_HESS_MAX_SLABS
#define TSG_HESS_MAX_SLABS 16
#endif
constexpr int kSlabRows = TSG_HESS_SLAB_ROWS;
constexpr int kMaxSlabs = TSG_HESS_MAX_SLABS;

__device__ inline double cabs1(c128 z) { return fabs(z.re) + fabs(z.im); }

__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Block-wide sum of doubles (blockDim.x == kEigThreads): wave reductions,
// then one pass over the per-wave partials.
__device__ double block_sum(double v, double* red) {
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  v = wave_sum(v);
  if (lane == 0) red[wv] = v;
  __syncthreads();
  double r = 0.0;
  for (int q = 0; q < kEigThreads / 64; ++q) r += red[q];
  __syncthreads();
  return r;
}

// ---------------------------------------------------------------- Hessenberg
// Householder reduction H <- P^H H P to upper Hessenberg form.  One column
// step applies P = I - beta v v^H from both sides in two sweeps over the
// trailing columns (P H P = H - beta v y - beta z v^H with y = v^H H,
// x = H v and z = x - beta (y v) v): the first sweep reads each element once
// for both products (wavefronts take rows, lanes take columns, so every load
// is coalesced; a lane keeps its columns' share of y and its columns' entries
// of v in registers), the second applies the rank-2 update.  That is half
// the matrix traffic of applying the two sides one after the other.  The
// reflectors are kept, v_k[1..] in column k of H below the subdiagonal (free
// once the column is reduced, so the working set stays one m x m matrix),
// beta_k and v_k[0] in rows 0 and 1 of R; the product Z = P_0 P_1 ... is
// formed afterwards by householder_z_kernel, many workgroups per matrix
// (each row of Z is transformed independently), and the Schur step clears
// the stored vectors from H.
template <int NQ, int RPI>
__global__ __launch_bounds__(kEigThreads) void hessenberg_kernel(c128* Hall, int64_t wsh, int m, c128* Rall,
                                                                 int64_t wsr, const int* __restrict__ wmap) {
  extern __shared__ c128 sm[];  // v[m], x[m], y[m], then NW x m partial y
  __shared__ double red[kEigThreads / 64];
  constexpr int NW = kEigThreads / 64;
  c128* v = sm;
  c128* xs = sm + m;
  c128* ys = sm + 2 * m;
  c128* yp = sm + 3 * m;
  const int w = wmap ? wmap[blockIdx.x] : blockIdx.x;
  if (w < 0) return;  // idle slot (whole workgroup)
  c128* H = Hall + int64_t(w) * wsh;
  c128* Rf = Rall + int64_t(w) * wsr;
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  for (int k = 0; k + 2 < m; ++k) {
    const int len = m - k - 1;  // rows k+1 .. m-1
    double part = 0.0;
    for (int i = t; i < len; i += kEigThreads) {
      const c128 x = H[int64_t(k + 1 + i) * m + k];
      v[i] = x;
      part += norm2(x);
    }
    const double alpha2 = block_sum(part, red);
    const c128 x0 = v[0];
    __syncthreads();  // every thread has read v[0] before it is rewritten
    const double ax0 = cabs(x0);
    const double alpha = sqrt(alpha2);
    if (alpha == 0.0 || alpha2 - ax0 * ax0 <= 1e-300 * (alpha2 > 0 ? alpha2 : 1.0)) {
      if (t == 0) Rf[k] = c128{0.0, 0.0};  // no reflector: beta = 0
      continue;
    }
    const c128 ph = ax0 > 0.0 ? c128{x0.re / ax0, x0.im / ax0} : c128{1.0, 0.0};
    if (t == 0) v[0] = x0 + alpha * ph;
    __syncthreads();
    const double beta = 1.0 / (alpha * (alpha + ax0));  // 2 / |v|^2
    if (t == 0) {
      Rf[k] = c128{beta, 0.0};
      Rf[int64_t(m) + k] = v[0];
    }
    const int ncols = m - k;  // columns k .. m-1 (column k + jj)
    // this lane's entries of v along the columns (v_e,j = v[jj - 1], jj >= 1)
    c128 vq[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      const int jj = lane + 64 * q;
      vq[q] = (jj >= 1 && jj < ncols) ? v[jj - 1] : c128{0.0, 0.0};
    }
    // sweep 1: x_i = sum_{j>k} H[i][j] v_e,j (all rows), y_j = sum_{i>k}
    // conj(v_e,i) H[i][j] (columns j >= k)
    c128 yacc[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) yacc[q] = c128{0.0, 0.0};
    for (int i0 = wv * RPI; i0 < m; i0 += NW * RPI) {
      c128 a[RPI][NQ];
#pragma unroll
      for (int r = 0; r < RPI; ++r) {
        const int i = i0 + r;
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
          const int jj = lane + 64 * q;
          a[r][q] = (i < m && jj < ncols) ? H[int64_t(i) * m + k + jj] : c128{0.0, 0.0};
        }
      }
#pragma unroll
      for (int r = 0; r < RPI; ++r) {
        const int i = i0 + r;
        c128 xr{0.0, 0.0};
        const c128 vi = (i > k && i < m) ? conj(v[i - k - 1]) : c128{0.0, 0.0};
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
          fma_acc(xr, a[r][q], vq[q]);
          fma_acc(yacc[q], vi, a[r][q]);
        }
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
          xr.re += __shfl_xor(xr.re, o, 64);
          xr.im += __shfl_xor(xr.im, o, 64);
        }
        if (lane == 0 && i < m) xs[i] = xr;
      }
    }
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      const int jj = lane + 64 * q;
      if (jj < ncols) yp[wv * m + jj] = yacc[q];
    }
    __syncthreads();
    // y (column sums over the wavefronts' partials) and s = y v_e
    double pr = 0.0, pi = 0.0;
    for (int jj = t; jj < ncols; jj += kEigThreads) {
      c128 y{0.0, 0.0};
      for (int q = 0; q < NW; ++q) y = y + yp[q * m + jj];
      ys[jj] = beta * y;
      if (jj >= 1) {
        const c128 vj = v[jj - 1];
        pr += y.re * vj.re - y.im * vj.im;
        pi += y.re * vj.im + y.im * vj.re;
      }
    }
    const double s_re = block_sum(pr, red), s_im = block_sum(pi, red);
    // z_i = beta (x_i - beta s v_e,i), over x
    for (int i = t; i < m; i += kEigThreads) {
      c128 z = xs[i];
      if (i > k) z = z - beta * (c128{s_re, s_im} * v[i - k - 1]);
      xs[i] = beta * z;
    }
    __syncthreads();
    // sweep 2: H[i][j] -= v_e,i (beta y_j) + (beta z_i) conj(v_e,j)
    c128 yq[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      const int jj = lane + 64 * q;
      yq[q] = jj < ncols ? ys[jj] : c128{0.0, 0.0};
      vq[q] = conj(vq[q]);
    }
    for (int i0 = wv * RPI; i0 < m; i0 += NW * RPI) {
      c128 a[RPI][NQ];
#pragma unroll
      for (int r = 0; r < RPI; ++r) {
        const int i = i0 + r;
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
          const int jj = lane + 64 * q;
          a[r][q] = (i < m && jj < ncols) ? H[int64_t(i) * m + k + jj] : c128{0.0, 0.0};
        }
      }
#pragma unroll
      for (int r = 0; r < RPI; ++r) {
        const int i = i0 + r;
        if (i >= m) continue;
        const c128 vi = i > k ? v[i - k - 1] : c128{0.0, 0.0};
        const c128 zi = xs[i];
        const c128 nvi{-vi.re, -vi.im}, nzi{-zi.re, -zi.im};
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
          const int jj = lane + 64 * q;
          c128 val = a[r][q];
          fma_acc(val, nvi, yq[q]);
          fma_acc(val, nzi, vq[q]);
          if (jj < ncols) H[int64_t(i) * m + k + jj] = val;
        }
      }
    }
    __syncthreads();
    for (int i = k + 2 + t; i < m; i += kEigThreads) H[int64_t(i) * m + k] = v[i - k - 1];
    __syncthreads();
  }
}

// The same reduction for larger bases, spread over several workgroups per
// matrix: the rows are cut into slabs, one workgroup each, and every column
// step is two launches (the launch boundary orders the slabs' accesses).
//   hess_slab_p: every workgroup forms the reflector from column k itself;
//     the first slab stores beta, v[0] and v; then each workgroup runs the
//     first sweep over its rows (x complete for its rows, a partial y).
//   hess_slab_u: each workgroup sums the partial ys, forms s and z for its
//     rows and applies the rank-2 update to them, then stores its share of
//     v below the subdiagonal of column k.
// Scratch in X beside the reflectors' scalars (rows 0 and 1): v in row 2, x
// in row 3, the partial ys in rows 4 .. 4 + nslab - 1.  With the grid laid
// out (window, slab), a window's slabs fall on one XCD when eight windows are
// batched, so its matrix stays in one L2.
template <int NQ, int RPI>
__global__ __launch_bounds__(kEigThreads) void hess_slab_p_kernel(const c128* Hall, int64_t wsh, int m, c128* Rall,
                                                                  int64_t wsr, int k, int rows,
                                                                  const int* __restrict__ wmap) {
  extern __shared__ c128 sm[];  // v[m], then NW x m partial y
  __shared__ double red[kEigThreads / 64];
  constexpr int NW = kEigThreads / 64;
  c128* v = sm;
  c128* yp = sm + m;
  const int w = wmap ? wmap[blockIdx.x] : blockIdx.x;
  if (w < 0) return;  // idle slot (whole workgroup)
  const int sl = int(blockIdx.y);
  const int r0 = sl * rows, r1 = min(m, r0 + rows);
  const c128* H = Hall + int64_t(w) * wsh;
  c128* Rf = Rall + int64_t(w) * wsr;
  c128* vbuf = Rf + 2 * int64_t(m);
  c128* xbuf = Rf + 3 * int64_t(m);
  c128* ypart = Rf + int64_t(4 + sl) * m;
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  const int len = m - k - 1;  // rows k+1 .. m-1
  double part = 0.0;
  for (int i = t; i < len; i += kEigThreads) {
    const c128 x = H[int64_t(k + 1 + i) * m + k];
    v[i] = x;
    part += norm2(x);
  }
  const double alpha2 = block_sum(part, red);
  const c128 x0 = v[0];
  __syncthreads();  // every thread has read v[0] before it is rewritten
  const double ax0 = cabs(x0);
  const double alpha = sqrt(alpha2);
  if (alpha == 0.0 || alpha2 - ax0 * ax0 <= 1e-300 * (alpha2 > 0 ? alpha2 : 1.0)) {
    if (sl == 0 && t == 0) Rf[k] = c128{0.0, 0.0};  // no reflector: beta = 0
    return;
  }
  const c128 ph = ax0 > 0.0 ? c128{x0.re / ax0, x0.im / ax0} : c128{1.0, 0.0};
  if (t == 0) v[0] = x0 + alpha * ph;
  __syncthreads();
  const double beta = 1.0 / (alpha * (alpha + ax0));  // 2 / |v|^2
  if (sl == 0) {
    if (t == 0) {
      Rf[k] = c128{beta, 0.0};
      Rf[int64_t(m) + k] = v[0];
    }
    for (int i = t; i < len; i += kEigThreads) vbuf[i] = v[i];
  }
  const int ncols = m - k;  // columns k .. m-1 (column k + jj)
  c128 vq[NQ];
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    const int jj = lane + 64 * q;
    vq[q] = (jj >= 1 && jj < ncols) ? v[jj - 1] : c128{0.0, 0.0};
  }
  c128 yacc[NQ];
#pragma unroll
  for (int q = 0; q < NQ; ++q) yacc[q] = c128{0.0, 0.0};
  for (int i0 = r0 + wv * RPI; i0 < r1; i0 += NW * RPI) {
    c128 a[RPI][NQ];
#pragma unroll
    for (int r = 0; r < RPI; ++r) {
      const int i = i0 + r;
#pragma unroll
      for (int q = 0; q < NQ; ++q) {
        const int jj = lane + 64 * q;
        a[r][q] = (i < r1 && jj < ncols) ? H[int64_t(i) * m + k + jj] : c128{0.0, 0.0};
      }
    }
#pragma unroll
    for (int r = 0; r < RPI; ++r) {
      const int i = i0 + r;
      c128 xr{0.0, 0.0};
      const c128 vi = (i > k && i < r1) ? conj(v[i - k - 1]) : c128{0.0, 0.0};
#pragma unroll
      for (int q = 0; q < NQ; ++q) {
        fma_acc(xr, a[r][q], vq[q]);
        fma_acc(yacc[q], vi, a[r][q]);
      }
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) {
        xr.re += __shfl_xor(xr.re, o, 64);
        xr.im += __shfl_xor(xr.im, o, 64);
      }
      if (lane == 0 && i < r1) xbuf[i] = xr;
    }
  }
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    const int jj = lane + 64 * q;
    if (jj < ncols) yp[wv * m + jj] = yacc[q];
  }
  __syncthreads();
  for (int jj = t; jj < ncols; jj += kEigThreads) {
    c128 y{0.0, 0.0};
    for (int q = 0; q < NW; ++q) y = y + yp[q * m + jj];
    ypart[jj] = y;
  }
}

template <int NQ, int RPI>
__global__ __launch_bounds__(kEigThreads) void hess_slab_u_kernel(c128* Hall, int64_t wsh, int m,
                                                                  const c128* __restrict__ Rall, int64_t wsr, int k,
                                                                  int rows, int nslab, const int* __restrict__ wmap) {
  extern __shared__ c128 sm[];  // v[m], beta y[m], beta z[rows]
  __shared__ double red[kEigThreads / 64];
  constexpr int NW = kEigThreads / 64;
  c128* v = sm;
  c128* ys = sm + m;
  c128* zs = sm + 2 * m;
  const int w = wmap ? wmap[blockIdx.x] : blockIdx.x;
  if (w < 0) return;  // idle slot (whole workgroup)
  const int sl = int(blockIdx.y);
  const int r0 = sl * rows, r1 = min(m, r0 + rows);
  c128* H = Hall + int64_t(w) * wsh;
  const c128* Rf = Rall + int64_t(w) * wsr;
  const double beta = Rf[k].re;
  if (beta == 0.0) return;  // uniform: no reflector at this column
  const c128* vbuf = Rf + 2 * int64_t(m);
  const c128* xbuf = Rf + 3 * int64_t(m);
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  const int len = m - k - 1, ncols = m - k;
  for (int i = t; i < len; i += kEigThreads) v[i] = vbuf[i];
  // y (sum of the slabs' partials) and s = y v_e
  double pr = 0.0, pi = 0.0;
  for (int jj = t; jj < ncols; jj += kEigThreads) {
    c128 y{0.0, 0.0};
    for (int q = 0; q < nslab; ++q) y = y + Rf[int64_t(4 + q) * m + jj];
    ys[jj] = beta * y;
    if (jj >= 1) {
      const c128 vj = vbuf[jj - 1];
      pr += y.re * vj.re - y.im * vj.im;
      pi += y.re * vj.im + y.im * vj.re;
    }
  }
  const double s_re = block_sum(pr, red), s_im = block_sum(pi, red);  // also orders v and ys
  for (int i = r0 + t; i < r1; i += kEigThreads) {
    c128 z = xbuf[i];
    if (i > k) z = z - beta * (c128{s_re, s_im} * v[i - k - 1]);
    zs[i - r0] = beta * z;
  }
  __syncthreads();
  c128 yq[NQ], vq[NQ];
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    const int jj = lane + 64 * q;
    yq[q] = jj < ncols ? ys[jj] : c128{0.0, 0.0};
    vq[q] = (jj >= 1 && jj < ncols) ? conj(v[jj - 1]) : c128{0.0, 0.0};
  }
  for (int i0 = r0 + wv * RPI; i0 < r1; i0 += NW * RPI) {
    c128 a[RPI][NQ];
#pragma unroll
    for (int r = 0; r < RPI; ++r) {
      const int i = i0 + r;
#pragma unroll
      for (int q = 0; q < NQ; ++q) {
        const int jj = lane + 64 * q;
        a[r][q] = (i < r1 && jj < ncols) ? H[int64_t(i) * m + k + jj] : c128{0.0, 0.0};
      }
    }
#pragma unroll
    for (int r = 0; r < RPI; ++r) {
      const int i = i0 + r;
      if (i >= r1) continue;
      const c128 vi = i > k ? v[i - k - 1] : c128{0.0, 0.0};
      const c128 zi = zs[i - r0];
      const c128 nvi{-vi.re, -vi.im}, nzi{-zi.re, -zi.im};
#pragma unroll
      for (int q = 0; q < NQ; ++q) {
        const int jj = lane + 64 * q;
        c128 val = a[r][q];
        fma_acc(val, nvi, yq[q]);
        fma_acc(val, nzi, vq[q]);
        if (jj < ncols) H[int64_t(i) * m + k + jj] = val;
      }
    }
  }
  __syncthreads();
  for (int i = max(k + 2, r0) + t; i < r1; i += kEigThreads) H[int64_t(i) * m + k] = v[i - k - 1];
}

// Z = P_0 P_1 ... P_{m-3} from the reflectors R of hessenberg_kernel, rows
// [r0, r0 + 16) per workgroup: each row starts as e_r and takes
// z[k+1..] -= beta_k (z[k+1..] v_k) v_k^H in order, sixteen lanes per row
// (the arithmetic of applying the reflectors to Z inside the reduction).
constexpr int kZRows = 16;

__global__ __launch_bounds__(kZRows * 16) void householder_z_kernel(const c128* __restrict__ Rall, int64_t wsr,
                                                                   const c128* __restrict__ Hall, int64_t wsh, int m,
                                                                   c128* Zall, int64_t wsz, int rows,
                                                                   const int* __restrict__ wmap) {
  extern __shared__ c128 zr[];  // rows x m (rows <= kZRows, blockDim = 16 rows)
  const int w = wmap ? wmap[blockIdx.y] : blockIdx.y;
  if (w < 0) return;
  const int r0 = int(blockIdx.x) * rows;
  if (r0 >= m) return;
  const c128* Rf = Rall + int64_t(w) * wsr;
  const c128* H = Hall + int64_t(w) * wsh;
  c128* Z = Zall + int64_t(w) * wsz;
  const int t = threadIdx.x, sub = t & 15, rr = t >> 4;
  const int r = r0 + rr;
  const bool ok = r < m;
  c128* row = zr + int64_t(rr) * m;
  for (int j = sub; j < m; j += 16) row[j] = c128{ok && j == r ? 1.0 : 0.0, 0.0};
  __syncthreads();
  for (int k = 0; k + 2 < m; ++k) {
    const double beta = Rf[k].re;
    if (beta == 0.0) continue;  // uniform: no reflector at this column
    const int len = m - k - 1;
    // v[0] in row 1 of R, v[j >= 1] in column k of H (row k + 1 + j)
    auto vj = [&](int j) { return j == 0 ? Rf[int64_t(m) + k] : H[int64_t(k + 1 + j) * m + k]; };
    double sr = 0.0, si = 0.0;
    for (int j = sub; j < len; j += 16) {
      const c128 a = row[k + 1 + j], b = vj(j);
      sr += a.re * b.re - a.im * b.im;
      si += a.re * b.im + a.im * b.re;
    }
#pragma unroll
    for (int o = 8; o > 0; o >>= 1) {
      sr += __shfl_xor(sr, o, 16);
      si += __shfl_xor(si, o, 16);
    }
    const c128 sc = beta * c128{sr, si};
    for (int j = sub; j < len; j += 16) {
      c128& h = row[k + 1 + j];
      h = h - sc * conj(vj(j));
    }
    __syncthreads();
  }
  if (ok)
    for (int j = sub; j < m; j += 16) Z[int64_t(r) * m + j] = row[j];
}

// ---------------------------------------------------------------- vectors
// X[:, j] = eigenvector of upper triangular T for T[j, j] (x_j = 1, x_i = 0
// for i > j), by back substitution.  One wavefront per eigenvector: each
// x_i needs the dot product of row i of T (contiguous) with the x_p already
// found, which the lanes split and reduce; x lives in LDS.
constexpr int kTrevcWaves = 4;

// Orders one wavefront's LDS traffic: its lanes run in lockstep and its LDS
// operations complete in order, so a fence plus a wave barrier suffices.
__device__ inline void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ inline c128 wave_sum(c128 v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    v.re += __shfl_xor(v.re, o, 64);
    v.im += __shfl_xor(v.im, o, 64);
  }
  return v;
}

__global__ __launch_bounds__(64 * kTrevcWaves) void trevc_kernel(const c128* Tall, int64_t wst, int m, c128* Xall,
                                                                 int64_t wsx, const int* __restrict__ wmap) {
  extern __shared__ c128 xs_all[];  // kTrevcWaves x m
  const int w = wmap ? wmap[blockIdx.y] : blockIdx.y;
  if (w < 0) return;  // idle slot (whole workgroup)
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int j = int(blockIdx.x) * kTrevcWaves + wv;
  if (j >= m) return;  // whole wavefront
  const c128* T = Tall + int64_t(w) * wst;
  c128* X = Xall + int64_t(w) * wsx;
  c128* xs = xs_all + int64_t(wv) * m;
  const c128 lam = T[int64_t(j) * m + j];
  double tnorm = 0.0;
  for (int i = lane; i < m; i += 64) tnorm = fmax(tnorm, cabs1(T[int64_t(i) * m + i]));
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) tnorm = fmax(tnorm, __shfl_xor(tnorm, o, 64));
  const double smin = fmax(2.220446049250313e-16 * tnorm, 1e-290);
  if (lane == 0) xs[j] = c128{1.0, 0.0};
  wave_lds_sync();
  for (int i = j - 1; i >= 0; --i) {
    const c128* Ti = T + int64_t(i) * m;
    c128 part{0.0, 0.0};
    for (int p = i + 1 + lane; p <= j; p += 64) fma_acc(part, Ti[p], xs[p]);
    const c128 sum = wave_sum(part);
    c128 d = Ti[i] - lam;
    if (cabs1(d) < smin) d = c128{smin, 0.0};
    const c128 xi = cdiv(c128{-sum.re, -sum.im}, d);
    if (lane == 0) xs[i] = xi;
    wave_lds_sync();
    if (cabs1(xi) > 1e150) {  // rescale to keep the back substitution finite
      for (int p = i + lane; p <= j; p += 64) xs[p] = 1e-150 * xs[p];
      wave_lds_sync();
    }
  }
  for (int p = lane; p < m; p += 64) X[int64_t(p) * m + j] = p <= j ? xs[p] : c128{0.0, 0.0};
}

// Y = Z X (m x m, row-major, 16 x 16 tiles), then each column of Y is
// normalised to unit 2-norm by colnorm_kernel.
__global__ __launch_bounds__(256) void small_gemm_kernel(const c128* Zall, int64_t wsz, const c128* Xall,
                                                         int64_t wsx, c128* Yall, int64_t wsy, int m,
                                                         const int* __restrict__ wmap) {
  __shared__ c128 As[16][17];
  __shared__ c128 Bs[16][17];
  const int w = wmap ? wmap[blockIdx.z] : blockIdx.z;
  if (w < 0) return;  // idle slot (whole workgroup)
  const c128* Z = Zall + int64_t(w) * wsz;
  const c128* X = Xall + int64_t(w) * wsx;
  c128* Y = Yall + int64_t(w) * wsy;
  const int tx = threadIdx.x % 16, ty = threadIdx.x / 16;
  const int i = blockIdx.y * 16 + ty, j = blockIdx.x * 16 + tx;
  c128 acc{0.0, 0.0};
  for (int k0 = 0; k0 < m; k0 += 16) {
    As[ty][tx] = (i < m && k0 + tx < m) ? Z[int64_t(i) * m + k0 + tx] : c128{0.0, 0.0};
    Bs[ty][tx] = (k0 + ty < m && j < m) ? X[int64_t(k0 + ty) * m + j] : c128{0.0, 0.0};
    __syncthreads();
#pragma unroll
    for (int k = 0; k < 16; ++k) fma_acc(acc, As[ty][k], Bs[k][tx]);
    __syncthreads();
  }
  if (i < m && j < m) Y[int64_t(i) * m + j] = acc;
}

__global__ void colnorm_kernel(c128* Yall, int64_t wsy, int m, const int* __restrict__ wmap) {
  const int w = wmap ? wmap[blockIdx.y] : blockIdx.y;
  if (w < 0) return;  // idle slot (whole workgroup)
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= m) return;
  c128* Y = Yall + int64_t(w) * wsy;
  double s = 0.0;
  for (int i = 0; i < m; ++i) s += norm2(Y[int64_t(i) * m + j]);
  const double f = s > 0.0 ? 1.0 / sqrt(s) : 1.0;
  for (int i = 0; i < m; ++i) Y[int64_t(i) * m + j] = f * Y[int64_t(i) * m + j];
}

// ---------------------------------------------------------------- selection
__device__ inline double sel_key(c128 th, c128 sigma, int mode) {
  if (mode == 1) return th.re;        // smallest real part
  if (mode == 2) return -th.re;       // largest real part
  return cabs(th - sigma);            // nearest the (complex) shift
}

__global__ __launch_bounds__(kSelThreads) void select_restart_kernel(const c128* thall, int64_t wst, const c128* Yall,
                                                             int64_t wsy, int m, const c128* sigma, int mode, int k,
                                                             int nev, c128* outall, int64_t wso, c128* thsel,
                                                             int64_t wss, const int* __restrict__ wmap) {
  extern __shared__ unsigned char smraw[];
  int* order = reinterpret_cast<int*>(smraw);                       // m
  c128* coef = reinterpret_cast<c128*>(smraw + ((m * sizeof(int) + 15) / 16) * 16);  // k * kSB
  c128* Wb = coef + size_t(k > 0 ? k : 1) * kSB;                                      // m * kSB
  __shared__ double red[kSelThreads];
  const int w = wmap ? wmap[blockIdx.x] : blockIdx.x;
  if (w < 0) return;  // idle slot (whole workgroup)
  const c128* th = thall + int64_t(w) * wst;
  const c128* Y = Yall + int64_t(w) * wsy;
  c128* out = outall + int64_t(w) * wso;
  const int ld = k + nev;
  const c128 sg = sigma ? sigma[w] : c128{0.0, 0.0};
  const int t = threadIdx.x;
  for (int i = t; i < m; i += kSelThreads) {
    const double ki = sel_key(th[i], sg, mode);
    int rank = 0;
    for (int j = 0; j < m; ++j) {
      const double kj = sel_key(th[j], sg, mode);
      bool before = (kj < ki) || (kj == ki && (th[j].re < th[i].re || (th[j].re == th[i].re &&
                    (th[j].im < th[i].im || (th[j].im == th[i].im && j < i)))));
      rank += before ? 1 : 0;
    }
    order[rank] = i;
  }
  __syncthreads();
  // nearest nev eigenvectors and their values
  for (int e = t; e < m * nev; e += kSelThreads) {
    const int i = e / nev, q = e % nev;
    out[int64_t(i) * ld + k + q] = Y[int64_t(i) * m + order[q]];
  }
  for (int q = t; q < nev; q += kSelThreads) thsel[int64_t(w) * wss + q] = th[order[q]];
  // orthonormal basis of the first k selected eigenvectors: blocks of kSB
  // columns staged in LDS, each made orthogonal to the columns before it by
  // two passes of block classical Gram-Schmidt, then orthonormalised inside
  // the block by two passes of classical Gram-Schmidt column by column
  for (int q0 = 0; q0 < k; q0 += kSB) {
    const int nb = min(kSB, k - q0);
    for (int e = t; e < m * kSB; e += kSelThreads) {
      const int i = e / kSB, j = e % kSB;
      Wb[e] = j < nb ? Y[int64_t(i) * m + order[q0 + j]] : c128{0.0, 0.0};
    }
    __syncthreads();
    for (int pass = 0; pass < 2 && q0 > 0; ++pass) {
      // C = out[:, :q0]^H W  (q0 x nb)
      for (int e = t; e < q0 * nb; e += kSelThreads) {
        const int p = e % q0, j = e / q0;
        // eight partial sums keep eight loads in flight
        c128 sp[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) sp[u] = c128{0.0, 0.0};
        int i = 0;
        for (; i + 7 < m; i += 8) {
          c128 a[8];
#pragma unroll
          for (int u = 0; u < 8; ++u) a[u] = out[int64_t(i + u) * ld + p];
#pragma unroll
          for (int u = 0; u < 8; ++u) fma_cacc(sp[u], a[u], Wb[(i + u) * kSB + j]);
        }
        for (; i < m; ++i) fma_cacc(sp[0], out[int64_t(i) * ld + p], Wb[i * kSB + j]);
        coef[p * kSB + j] = ((sp[0] + sp[1]) + (sp[2] + sp[3])) + ((sp[4] + sp[5]) + (sp[6] + sp[7]));
      }
      __syncthreads();
      // W -= out[:, :q0] C, one thread per row
      for (int i = t; i < m; i += kSelThreads) {
        c128 acc[kSB];
#pragma unroll
        for (int j = 0; j < kSB; ++j) acc[j] = c128{0.0, 0.0};
        const c128* row = out + int64_t(i) * ld;
        int p = 0;
        for (; p + 3 < q0; p += 4) {
          c128 a[4];
#pragma unroll
          for (int u = 0; u < 4; ++u) a[u] = row[p + u];
#pragma unroll
          for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int j = 0; j < kSB; ++j) fma_acc(acc[j], a[u], coef[(p + u) * kSB + j]);
        }
        for (; p < q0; ++p) {
          const c128 a = row[p];
#pragma unroll
          for (int j = 0; j < kSB; ++j) fma_acc(acc[j], a, coef[p * kSB + j]);
        }
#pragma unroll
        for (int j = 0; j < kSB; ++j) Wb[i * kSB + j] = Wb[i * kSB + j] - acc[j];
      }
      __syncthreads();
    }
    for (int q = 0; q < nb; ++q) {
      for (int pass = 0; pass < 2 && q > 0; ++pass) {
        if (t < q) {
          c128 s{0.0, 0.0};
          for (int i = 0; i < m; ++i) fma_cacc(s, Wb[i * kSB + t], Wb[i * kSB + q]);
          coef[t] = s;
        }
        __syncthreads();
        for (int i = t; i < m; i += kSelThreads) {
          c128 v = Wb[i * kSB + q];
          for (int p = 0; p < q; ++p) v = v - Wb[i * kSB + p] * coef[p];
          Wb[i * kSB + q] = v;
        }
        __syncthreads();
      }
      double part = 0.0;
      for (int i = t; i < m; i += kSelThreads) part += norm2(Wb[i * kSB + q]);
      red[t] = part;
      __syncthreads();
      for (int o = kSelThreads / 2; o > 0; o >>= 1) {
        if (t < o) red[t] += red[t + o];
        __syncthreads();
      }
      const double nrm = sqrt(red[0]);
      __syncthreads();
      const double f = nrm > 0.0 ? 1.0 / nrm : 0.0;
      for (int i = t; i < m; i += kSelThreads) Wb[i * kSB + q] = f * Wb[i * kSB + q];
      __syncthreads();
    }
    for (int e = t; e < m * nb; e += kSelThreads) {
      const int i = e / nb, j = e % nb;
      out[int64_t(i) * ld + q0 + j] = Wb[i * kSB + j];
    }
    __syncthreads();
  }
}

}  // namespace

int64_t smalleig_workspace(int m) { return 2 * int64_t(m) * m + schur_log_size(m); }

void smalleig(c128* H, int64_t wsh, int m, c128* theta, int64_t wst, c128* Y, int64_t wsy, c128* work, int64_t wsw,
              int* info, int nwin, hipStream_t st, const int* wmap) {
  if (nwin <= 0 || m <= 0) return;
  c128* Z = work;               // m*m per window at stride wsw
  c128* X = work + int64_t(m) * m;
  // the reflectors' scalars go to X, which is free until the eigenvector step
  const size_t hlds = size_t(3 + kEigThreads / 64) * m * sizeof(c128);
  if (hlds > size_t(150) * 1024) throw DeviceError("hessenberg: basis too large for the LDS");
  auto hess = [&](auto kern) {
    if (hlds > size_t(64) * 1024) {
      static size_t granted = 0;
      if (hlds > granted) {
        const hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                                 hipFuncAttributeMaxDynamicSharedMemorySize, int(hlds));
        if (e != hipSuccess) throw DeviceError(std::string("hessenberg: LDS attribute: ") + hipGetErrorString(e));
        granted = hlds;
      }
    }
    hipLaunchKernelGGL(kern, dim3(nwin), dim3(kEigThreads), hlds, st, H, wsh, m, X, wsw, wmap);
  };
  if (m > kMaxDenseBasis) throw DeviceError("hessenberg: basis too large");
  if (m < kSlabMinBasis) {
    if (m <= 8 * 64)
      hess(hessenberg_kernel<8, 2>);
    else
      hess(hessenberg_kernel<14, 1>);
  } else {
    // about kSlabRows rows per slab, at most kMaxSlabs slabs
    int nslab = std::min(kMaxSlabs, (m + kSlabRows - 1) / kSlabRows);
    const int rows = (m + nslab - 1) / nslab;
    nslab = (m + rows - 1) / rows;
    if (int64_t(4 + nslab) * m > int64_t(m) * m) throw DeviceError("hessenberg: scratch does not fit in X");
    const size_t plds = size_t(1 + kEigThreads / 64) * m * sizeof(c128);
    const size_t ulds = size_t(2 * m + rows) * sizeof(c128);
    if (plds > size_t(150) * 1024) throw DeviceError("hessenberg: basis too large for the LDS");
    auto slabs = [&](auto pk, auto uk) {
      if (plds > size_t(64) * 1024) {
        static size_t granted = 0;
        if (plds > granted) {
          const hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(pk),
                                                   hipFuncAttributeMaxDynamicSharedMemorySize, int(plds));
          if (e != hipSuccess) throw DeviceError(std::string("hessenberg: LDS attribute: ") + hipGetErrorString(e));
          granted = plds;
        }
      }
      const dim3 grid{unsigned(nwin), unsigned(nslab), 1u};
      for (int k = 0; k + 2 < m; ++k) {
        hipLaunchKernelGGL(pk, grid, dim3(kEigThreads), plds, st, H, wsh, m, X, wsw, k, rows, wmap);
        hipLaunchKernelGGL(uk, grid, dim3(kEigThreads), ulds, st, H, wsh, m, X, wsw, k, rows, nslab, wmap);
      }
    };
    if (m <= 8 * 64)
      slabs(hess_slab_p_kernel<8, 2>, hess_slab_u_kernel<8, 2>);
    else
      slabs(hess_slab_p_kernel<14, 1>, hess_slab_u_kernel<14, 1>);
  }
  const int zrows = int(std::max<size_t>(1, std::min<size_t>(kZRows, (size_t(150) * 1024) / (size_t(m) * sizeof(c128)))));
  const size_t zlds = size_t(zrows) * m * sizeof(c128);
  if (zlds > size_t(150) * 1024) throw DeviceError("householder_z: basis too large for the LDS");
  if (zlds > size_t(64) * 1024) {
    static size_t granted = 0;
    if (zlds > granted) {
      const hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(householder_z_kernel),
                                               hipFuncAttributeMaxDynamicSharedMemorySize, int(zlds));
      if (e != hipSuccess) throw DeviceError(std::string("householder_z: LDS attribute: ") + hipGetErrorString(e));
      granted = zlds;
    }
  }
  hipLaunchKernelGGL(householder_z_kernel, dim3((m + zrows - 1) / zrows, nwin), dim3(zrows * 16), zlds, st, X, wsw,
                     H, wsh, m, Z, wsw, zrows, wmap);
  launch_schur(H, wsh, m, Z, wsw, work + 2 * int64_t(m) * m, wsw, theta, wst, info, nwin, st, wmap);
  const size_t tlds = size_t(kTrevcWaves) * m * sizeof(c128);
  if (tlds > size_t(150) * 1024) throw DeviceError("trevc: basis too large for the LDS");
  if (tlds > size_t(64) * 1024) {
    static size_t granted = 0;
    if (tlds > granted) {
      const hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(trevc_kernel),
                                               hipFuncAttributeMaxDynamicSharedMemorySize, int(tlds));
      if (e != hipSuccess) throw DeviceError(std::string("trevc: LDS attribute: ") + hipGetErrorString(e));
      granted = tlds;
    }
  }
  hipLaunchKernelGGL(trevc_kernel, dim3((m + kTrevcWaves - 1) / kTrevcWaves, nwin), dim3(64 * kTrevcWaves), tlds, st,
                     H, wsh, m, X, wsw, wmap);
  hipLaunchKernelGGL(small_gemm_kernel, dim3((m + 15) / 16, (m + 15) / 16, nwin), dim3(256), 0, st, Z, wsw, X, wsw,
                     Y, wsy, m, wmap);
  hipLaunchKernelGGL(colnorm_kernel, dim3((m + 63) / 64, nwin), dim3(64), 0, st, Y, wsy, m, wmap);
}

void select_restart(const c128* theta, int64_t wst, const c128* Y, int64_t wsy, int m, const c128* sigma, int mode,
                    int k, int nev, c128* out, int64_t wso, c128* theta_sel, int64_t wss, int nwin, hipStream_t st,
                    const int* wmap) {
  if (nwin <= 0) return;
  const size_t smem = ((m * sizeof(int) + 15) / 16) * 16 + size_t(std::max(k, 1) + m) * kSB * sizeof(c128);
  // beyond the default 64 KiB the kernel must be allowed more dynamic LDS
  // (its static part is 4 KiB of the 160 KiB)
  if (smem > size_t(150) * 1024) throw DeviceError("select_restart: basis too large for the LDS");
  if (smem > size_t(64) * 1024) {
    static size_t granted = 0;
    if (smem > granted) {
      const hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(select_restart_kernel),
                                               hipFuncAttributeMaxDynamicSharedMemorySize, int(smem));
      if (e != hipSuccess) throw DeviceError(std::string("select_restart: LDS attribute: ") + hipGetErrorString(e));
      granted = smem;
    }
  }
  hipLaunchKernelGGL(select_restart_kernel, dim3(nwin), dim3(kSelThreads), smem, st, theta, wst, Y, wsy, m, sigma, mode, k,
                     nev, out, wso, theta_sel, wss, wmap);
}

}  // namespace tsg
