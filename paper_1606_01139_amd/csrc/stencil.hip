// K1: block matrix-vector product Y = A X for the real-space operator
//   A = -1/2 Lap_h + V(r) - i (Gamma_L + Gamma_R)(z)
// (Eq. (1) of Feldman & Zhou; Section 1: the operator is applied only as a
// matrix-vector product formula).  The Laplacian is the radius-R central
// difference star (2R+1 taps per axis, 6R+1 in all) with zero values outside
// the box.
//
// Layout: a block of B vectors is stored point-major, X[n * ld + c] for grid
// point n = x + nx (y + ny z) and column c < B, so one point's B values are
// contiguous.  Batched over windows: blockIdx.z selects a window whose block
// sits at a fixed element stride from the previous one.
//
// Mapping: one thread owns one (x, y, column) and walks a chunk of z planes;
// the 2R+1 z-neighbours live in a register queue (each input value is loaded
// once per z-walk), x- and y-neighbours are read through L1/L2.
#include "kernels.h"

namespace tsg {

template <typename T, int R>
__global__ __launch_bounds__(256) void stencil_kernel(StencilArgs<T> a) {
  const int w = a.wmap ? a.wmap[blockIdx.z] : blockIdx.z;
  const int64_t gid = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  const int nc = a.ncols;
  const int64_t plane = int64_t(a.nx) * a.ny;
  if (gid >= plane * nc) return;
  const int c = int(gid % nc);
  const int64_t xy = gid / nc;
  const int x = int(xy % a.nx);
  const int y = int(xy / a.nx);
  const int z0 = blockIdx.y * a.zchunk;
  const int z1 = min(a.nz, z0 + a.zchunk);
  if (z0 >= z1) return;

  const cplx<T>* __restrict__ X = a.X + int64_t(w) * a.wsx + c;
  cplx<T>* __restrict__ Y = a.Y + int64_t(w) * a.wsy + c;
  const int64_t ldx = a.ldx;
  const T shift = a.shifts ? a.shifts[w] : T(0);

  // z register queue: q[j] holds the value at plane z - R + j
  cplx<T> q[2 * R + 1];
#pragma unroll
  for (int j = 0; j < 2 * R + 1; ++j) {
    int zz = z0 - R + j;
    q[j] = (zz >= 0 && zz < a.nz) ? X[(zz * plane + xy) * ldx] : cplx<T>{T(0), T(0)};
  }
  for (int z = z0; z < z1; ++z) {
    const int64_t n = z * plane + xy;
    const cplx<T>* __restrict__ Xp = X + n * ldx;
    cplx<T> acc = q[R];
    const T d = a.diag0 + a.V[n] - shift;
    const T gi = -a.gamma[z];
    acc = cplx<T>{d * acc.re - gi * acc.im, d * acc.im + gi * acc.re};
#pragma unroll
    for (int m = 1; m <= R; ++m) {
      const T cm = a.coef[m];
      cplx<T> s = q[R - m] + q[R + m];
      if (x - m >= 0) s = s + Xp[-int64_t(m) * ldx];
      if (x + m < a.nx) s = s + Xp[int64_t(m) * ldx];
      if (y - m >= 0) s = s + Xp[-int64_t(m) * a.nx * ldx];
      if (y + m < a.ny) s = s + Xp[int64_t(m) * a.nx * ldx];
      acc.re = fma(cm, s.re, acc.re);
      acc.im = fma(cm, s.im, acc.im);
    }
    Y[n * a.ldy] = acc;
    // advance the queue
#pragma unroll
    for (int j = 0; j < 2 * R; ++j) q[j] = q[j + 1];
    const int zn = z + R + 1;
    q[2 * R] = (zn < a.nz) ? X[(zn * plane + xy) * ldx] : cplx<T>{T(0), T(0)};
  }
}

template <typename T>
void launch_stencil(const StencilArgs<T>& a, int nwin, hipStream_t s) {
  if (nwin <= 0 || a.ncols <= 0) return;
  const int64_t threads = int64_t(a.nx) * a.ny * a.ncols;
  dim3 block(256);
  dim3 grid(unsigned((threads + 255) / 256), unsigned((a.nz + a.zchunk - 1) / a.zchunk), unsigned(nwin));
  switch (a.radius) {
    case 1: hipLaunchKernelGGL((stencil_kernel<T, 1>), grid, block, 0, s, a); break;
    case 2: hipLaunchKernelGGL((stencil_kernel<T, 2>), grid, block, 0, s, a); break;
    case 3: hipLaunchKernelGGL((stencil_kernel<T, 3>), grid, block, 0, s, a); break;
    case 4: hipLaunchKernelGGL((stencil_kernel<T, 4>), grid, block, 0, s, a); break;
    case 5: hipLaunchKernelGGL((stencil_kernel<T, 5>), grid, block, 0, s, a); break;
    default: hipLaunchKernelGGL((stencil_kernel<T, 6>), grid, block, 0, s, a); break;
  }
}

template void launch_stencil<double>(const StencilArgs<double>&, int, hipStream_t);
template void launch_stencil<float>(const StencilArgs<float>&, int, hipStream_t);

}  // namespace tsg
