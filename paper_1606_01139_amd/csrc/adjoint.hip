// Adjoint of L = sum_e w_e T(E_e) (T of Section 1 built from the combined
// eigenpairs) with respect to V(r) and the absorber parameters.  The paper
// does not differentiate T; the derivative here is that of the computed
// quantity with the energies held fixed.
//
// With c-normalised pairs (u^T u = 1), g_k(E) = 1/(E - eps_k),
// M^X = U^T Gamma_X conj(U) and dA = diag(dV) - i diag(dGamma):
//   d eps_k = u_k^T dA u_k  (first-order perturbation of Eq. (5)'s kind),
//   d u_k   = sum_{j != k} u_j (u_j^T dA u_k) / (eps_k - eps_j),
// and dL = 2 Re sum_k mu_k^T dA u_k + (explicit Gamma terms), where
//   mu_k = sum_{j in S} u_j B_jk + lambda_k.
// Summed over the computed set the in-set eigenvector terms telescope with
// the eigenvalue terms: the pair (j, k) contributes through
// (g_k - g_j)/(eps_k - eps_j) = g_j g_k, so the in-set part of dG is
// G dA G and needs no eigenvalue difference (finite at degeneracy):
//   B = (P + P^T)/2,  P_jk = sum_e w_e g_j g_k sum_l conj(g_l) M^R_jl M^L_kl.
// The out-of-set part:
//   z_k  = Gamma_R conj(U) (K^R)^T e_k + Gamma_L conj(U) (K^L)^T e_k,
//   K^R  = Q o M^L, K^L = Q o M^R, Q_kl = sum_e w_e g_k conj(g_l),
//   lambda_k solves (eps_k - A) lambda_k = (I - U U^T) z_k in the
//   complement of the computed set (projected COCR, all k at once).
// The explicit dependence of T on Gamma_X gives
//   D_X(r) = Re sum_k u_k(r) (conj(U) (K^X)^T)_{r k}.
// Small n x n and n x nE quantities are formed by simple kernels; the N-long
// work uses the batched products of dense.hip and the stencil.
#include <algorithm>

#include "kernels.h"

namespace tsg {
namespace {

__global__ void gmat_kernel(const c128* eps, int n, const double* E, int nE, c128* G) {
  const int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= int64_t(n) * nE) return;
  const int k = int(e / nE), q = int(e % nE);
  G[e] = cdiv(c128{1.0, 0.0}, c128{E[q] - eps[k].re, -eps[k].im});
}

// Q_kl = sum_e w_e g_k conj(g_l);  KRt[l][k] = Q_kl ML_kl, KLt[l][k] = Q_kl MR_kl
__global__ void kmat_kernel(const c128* G, int n, int nE, const double* w, const c128* MR, const c128* ML,
                            c128* KRt, c128* KLt) {
  const int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= int64_t(n) * n) return;
  const int k = int(e / n), l = int(e % n);
  c128 q{0.0, 0.0};
  for (int t = 0; t < nE; ++t) fma_acc(q, w[t] * G[int64_t(k) * nE + t], conj(G[int64_t(l) * nE + t]));
  KRt[int64_t(l) * n + k] = q * ML[e];
  KLt[int64_t(l) * n + k] = q * MR[e];
}

// P_jk = sum_e w_e g_j(e) g_k(e) sum_l conj(g_l(e)) MR_jl ML_kl: a product
// whose contraction index runs over (energy, l), with the factors formed
// while the MR and ML tiles are staged in LDS.  Tiles of 32 x 32 outputs,
// 256 threads, 2 x 2 outputs per thread.
constexpr int kPT = 32, kPL = 16;
__global__ __launch_bounds__(256) void pmat_kernel(const c128* __restrict__ G, int n, int nE,
                                                   const double* __restrict__ w, const c128* __restrict__ MR,
                                                   const c128* __restrict__ ML, c128* __restrict__ P) {
  __shared__ c128 a[kPL][kPT + 1];  // conj(g_l) MR_jl, [l][j]
  __shared__ c128 b[kPL][kPT + 1];  // ML_kl, [l][k]
  __shared__ c128 gj[kPT], gk[kPT];
  const int j0 = blockIdx.y * kPT, k0 = blockIdx.x * kPT;
  const int tx = threadIdx.x % 16, ty = threadIdx.x / 16;  // outputs (j0 + 2ty + p, k0 + 2tx + q)
  c128 acc[2][2] = {};
  for (int e = 0; e < nE; ++e) {
    __syncthreads();
    if (threadIdx.x < kPT) {
      const int j = j0 + threadIdx.x;
      gj[threadIdx.x] = j < n ? G[int64_t(j) * nE + e] : c128{0.0, 0.0};
    } else if (threadIdx.x < 2 * kPT) {
      const int k = k0 + threadIdx.x - kPT;
      gk[threadIdx.x - kPT] = k < n ? G[int64_t(k) * nE + e] : c128{0.0, 0.0};
    }
    c128 t[2][2] = {};
    for (int l0 = 0; l0 < n; l0 += kPL) {
      __syncthreads();
      for (int i = threadIdx.x; i < kPL * kPT; i += 256) {
        const int li = i % kPL, ri = i / kPL;
        const int l = l0 + li;
        const int j = j0 + ri, k = k0 + ri;
        c128 av{0.0, 0.0}, bv{0.0, 0.0};
        if (l < n) {
          const c128 gl = conj(G[int64_t(l) * nE + e]);
          if (j < n) av = gl * MR[int64_t(j) * n + l];
          if (k < n) bv = ML[int64_t(k) * n + l];
        }
        a[li][ri] = av;
        b[li][ri] = bv;
      }
      __syncthreads();
#pragma unroll 4
      for (int li = 0; li < kPL; ++li) {
        const c128 a0 = a[li][2 * ty], a1 = a[li][2 * ty + 1];
        const c128 b0 = b[li][2 * tx], b1 = b[li][2 * tx + 1];
        fma_acc(t[0][0], a0, b0); fma_acc(t[0][1], a0, b1);
        fma_acc(t[1][0], a1, b0); fma_acc(t[1][1], a1, b1);
      }
    }
    const double we = w[e];
#pragma unroll
    for (int p = 0; p < 2; ++p)
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        const c128 s = we * (gj[2 * ty + p] * gk[2 * tx + q]);
        fma_acc(acc[p][q], s, t[p][q]);
      }
  }
#pragma unroll
  for (int p = 0; p < 2; ++p)
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const int j = j0 + 2 * ty + p, k = k0 + 2 * tx + q;
      if (j < n && k < n) P[int64_t(j) * n + k] = acc[p][q];
    }
}

// B = (P + P^T) / 2
__global__ void symmetrize_kernel(const c128* P, int n, c128* B) {
  const int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= int64_t(n) * n) return;
  const int j = int(e / n), k = int(e % n);
  B[e] = 0.5 * (P[e] + P[int64_t(k) * n + j]);
}

__global__ void conj_kernel(const c128* X, c128* Y, int64_t total) {
  const int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e < total) Y[e] = conj(X[e]);
}

// Z = gR o YR + gL o YL (per grid row; gamma depends on the z plane)
__global__ void zcombine_kernel(const c128* YR, const c128* YL, const double* gR, const double* gL, int64_t N, int n,
                                int64_t plane, c128* Z) {
  const int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= N * n) return;
  const int64_t r = e % N;
  const int64_t z = r / plane;
  Z[e] = gR[z] * YR[e] + gL[z] * YL[e];
}

// out[r] += scale * Re sum_k U[r,k] Y[r,k]  (or Im with use_im)
__global__ void rowdot_kernel(const c128* U, const c128* Y, int64_t N, int n, double scale, int use_im, double* out) {
  const int64_t r = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (r >= N) return;
  c128 s{0.0, 0.0};
  for (int k = 0; k < n; ++k) fma_acc(s, U[int64_t(k) * N + r], Y[int64_t(k) * N + r]);
  out[r] += scale * (use_im ? s.im : s.re);
}

// ---------------------------------------------------------------- COCR
// Per-column sums over rows (deterministic two-pass): for each column k,
// {r^T s (complex), p^T p (complex), |r|^2}.
constexpr int kCC = 256;
__global__ __launch_bounds__(kCC) void cocr_partial(const c128* R, const c128* S, const c128* P, int64_t N, int n,
                                                    int nchunk, double* part) {
  __shared__ double red[5][kCC / 64];
  const int k = blockIdx.y, chunk = blockIdx.x;
  const int64_t per = (N + nchunk - 1) / nchunk;
  const int64_t n0 = chunk * per, n1 = min(N, n0 + per);
  c128 rs{0.0, 0.0}, pp{0.0, 0.0};
  double rr = 0.0;
  const c128* r = R + int64_t(k) * N;
  const c128* s = S + int64_t(k) * N;
  const c128* p = P + int64_t(k) * N;
  for (int64_t i = n0 + threadIdx.x; i < n1; i += kCC) {
    const c128 a = r[i];
    fma_acc(rs, a, s[i]);
    fma_acc(pp, p[i], p[i]);
    rr += norm2(a);
  }
  double v[5] = {rs.re, rs.im, pp.re, pp.im, rr};
  const int lane = threadIdx.x % 64, wv = threadIdx.x / 64;
#pragma unroll
  for (int q = 0; q < 5; ++q) {
    double x = v[q];
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
    if (lane == 0) red[q][wv] = x;
  }
  __syncthreads();
  if (threadIdx.x < 5) {
    double x = 0.0;
    for (int q = 0; q < kCC / 64; ++q) x += red[threadIdx.x][q];
    part[(int64_t(chunk) * n + k) * 5 + threadIdx.x] = x;
  }
}

__global__ void cocr_reduce(const double* part, int nchunk, int n, double* out) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n * 5) return;
  double x = 0.0;
  for (int c = 0; c < nchunk; ++c) x += part[int64_t(c) * n * 5 + e];
  out[e] = x;
}

// M_k r = eps_k r - A r  (A r already in AR)
__global__ void shift_kernel(const c128* R, c128* AR, const c128* eps, int64_t N, int n) {
  const int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= N * n) return;
  const int k = int(e / N);
  AR[e] = eps[k] * R[e] - AR[e];
}

// step scalars from the sums: mode 0 (start) rho = r^T M r;
// mode 1: alpha = rho / (Mp)^T (Mp); mode 2: beta = rho_new / rho, rho = rho_new.
__global__ void cocr_scalars(const double* sums, int n, int mode, c128* rho, c128* alpha, c128* beta, int* done) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const c128 rs{sums[k * 5 + 0], sums[k * 5 + 1]};
  if (mode == 0) {
    rho[k] = rs;
  } else if (mode == 1) {
    const c128 pp{sums[k * 5 + 2], sums[k * 5 + 3]};
    const bool ok = !done[k] && (pp.re != 0.0 || pp.im != 0.0);
    alpha[k] = ok ? cdiv(rho[k], pp) : c128{0.0, 0.0};
  } else {
    const bool ok = !done[k] && (rho[k].re != 0.0 || rho[k].im != 0.0);
    beta[k] = ok ? cdiv(rs, rho[k]) : c128{0.0, 0.0};
    rho[k] = rs;
  }
}

// x += alpha p; r -= alpha Mp
__global__ void cocr_xr(c128* X, c128* R, const c128* P, const c128* MP, const c128* alpha, int64_t N, int n) {
  const int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= N * n) return;
  const c128 a = alpha[e / N];
  X[e] = X[e] + a * P[e];
  R[e] = R[e] - a * MP[e];
}

// p = r + beta p; Mp = Mr + beta Mp
__global__ void cocr_p(c128* P, c128* MP, const c128* R, const c128* MR, const c128* beta, int64_t N, int n) {
  const int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= N * n) return;
  const c128 b = beta[e / N];
  P[e] = R[e] + b * P[e];
  MP[e] = MR[e] + b * MP[e];
}

__global__ void add_kernel(c128* Y, const c128* X, int64_t total) {
  const int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e < total) Y[e] = Y[e] + X[e];
}

// dabs[p] = sum_r dGamma_side(p)(r) * prof_p(z(r)); one workgroup per parameter
__global__ __launch_bounds__(256) void absorber_kernel(const double* dGL, const double* dGR, const double* prof,
                                                       int64_t N, int nz, int64_t plane, double* out) {
  __shared__ double red[256];
  const int p = blockIdx.x;
  const double* d = (p < 2) ? dGL : dGR;
  double s = 0.0;
  for (int64_t r = threadIdx.x; r < N; r += 256) s += d[r] * prof[int64_t(p) * nz + r / plane];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[p] = red[0];
}

inline unsigned blocks(int64_t total, int t = 256) { return unsigned((total + t - 1) / t); }

}  // namespace

void adj_gmat(const c128* eps, int n, const double* E, int nE, c128* G, hipStream_t st) {
  hipLaunchKernelGGL(gmat_kernel, dim3(blocks(int64_t(n) * nE)), dim3(256), 0, st, eps, n, E, nE, G);
}
void adj_kmats(const c128* G, int n, int nE, const double* w, const c128* MR, const c128* ML, c128* KRt, c128* KLt,
               hipStream_t st) {
  hipLaunchKernelGGL(kmat_kernel, dim3(blocks(int64_t(n) * n)), dim3(256), 0, st, G, n, nE, w, MR, ML, KRt, KLt);
}
void adj_inset(const c128* G, int n, int nE, const double* w, const c128* MR, const c128* ML, c128* P, c128* B,
               hipStream_t st) {
  const unsigned t = unsigned((n + kPT - 1) / kPT);
  hipLaunchKernelGGL(pmat_kernel, dim3(t, t), dim3(256), 0, st, G, n, nE, w, MR, ML, P);
  hipLaunchKernelGGL(symmetrize_kernel, dim3(blocks(int64_t(n) * n)), dim3(256), 0, st, P, n, B);
}
void adj_conj(const c128* X, c128* Y, int64_t total, hipStream_t st) {
  hipLaunchKernelGGL(conj_kernel, dim3(blocks(total)), dim3(256), 0, st, X, Y, total);
}
void adj_zcombine(const c128* YR, const c128* YL, const double* gR, const double* gL, int64_t N, int n,
                  int64_t plane, c128* Z, hipStream_t st) {
  hipLaunchKernelGGL(zcombine_kernel, dim3(blocks(N * n)), dim3(256), 0, st, YR, YL, gR, gL, N, n, plane, Z);
}
void adj_rowdot(const c128* U, const c128* Y, int64_t N, int n, double scale, bool use_im, double* out,
                hipStream_t st) {
  hipLaunchKernelGGL(rowdot_kernel, dim3(blocks(N)), dim3(256), 0, st, U, Y, N, n, scale, use_im ? 1 : 0, out);
}
int64_t adj_cocr_workspace(int64_t N, int n) {
  const int64_t nchunk = std::max<int64_t>(1, std::min<int64_t>((N + 4095) / 4096, 64));
  return nchunk * n * 5;
}
void adj_cocr_sums(const c128* R, const c128* S, const c128* P, int64_t N, int n, double* part, double* out,
                   hipStream_t st) {
  const int nchunk = int(std::max<int64_t>(1, std::min<int64_t>((N + 4095) / 4096, 64)));
  hipLaunchKernelGGL(cocr_partial, dim3(nchunk, n), dim3(kCC), 0, st, R, S, P, N, n, nchunk, part);
  hipLaunchKernelGGL(cocr_reduce, dim3(blocks(int64_t(n) * 5)), dim3(256), 0, st, part, nchunk, n, out);
}
void adj_shift(const c128* R, c128* AR, const c128* eps, int64_t N, int n, hipStream_t st) {
  hipLaunchKernelGGL(shift_kernel, dim3(blocks(N * n)), dim3(256), 0, st, R, AR, eps, N, n);
}
void adj_scalars(const double* sums, int n, int mode, c128* rho, c128* alpha, c128* beta, int* done,
                 hipStream_t st) {
  hipLaunchKernelGGL(cocr_scalars, dim3(blocks(n, 64)), dim3(64), 0, st, sums, n, mode, rho, alpha, beta, done);
}
void adj_xr(c128* X, c128* R, const c128* P, const c128* MP, const c128* alpha, int64_t N, int n, hipStream_t st) {
  hipLaunchKernelGGL(cocr_xr, dim3(blocks(N * n)), dim3(256), 0, st, X, R, P, MP, alpha, N, n);
}
void adj_p(c128* P, c128* MP, const c128* R, const c128* MR, const c128* beta, int64_t N, int n, hipStream_t st) {
  hipLaunchKernelGGL(cocr_p, dim3(blocks(N * n)), dim3(256), 0, st, P, MP, R, MR, beta, N, n);
}
void adj_add(c128* Y, const c128* X, int64_t total, hipStream_t st) {
  hipLaunchKernelGGL(add_kernel, dim3(blocks(total)), dim3(256), 0, st, Y, X, total);
}
void adj_absorber(const double* dGL, const double* dGR, const double* prof, int64_t N, int nz, int64_t plane,
                  double* out, hipStream_t st) {
  hipLaunchKernelGGL(absorber_kernel, dim3(4), dim3(256), 0, st, dGL, dGR, prof, N, nz, plane, out);
}

}  // namespace tsg
