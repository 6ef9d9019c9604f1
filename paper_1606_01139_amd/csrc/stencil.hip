// K1: block matrix-vector product Y = A X for the real-space operator
//   A = -1/2 Lap_h + V(r) - i (Gamma_L + Gamma_R)(z)
// (Eq. (1) of Feldman & Zhou; Section 1: the operator is applied only as a
// matrix-vector product formula).  The Laplacian is the radius-R central
// difference star (2R+1 taps per axis, 6R+1 in all) with zero values outside
// the box.
//
// Layout: each vector is one contiguous grid function, X[n] with
// n = x + nx (y + ny z).  A launch covers every column of every active window
// (blockIdx.z = slot * ncols + column); windows may belong to different
// systems, each described by a SysDesc.
//
// Mapping (2.5-D blocking): a workgroup owns a tx x ty tile of one xy plane
// and walks a chunk of z planes.  Each thread keeps its point's 2R+1 z
// neighbours in a register queue, so every interior value is read from HBM
// once per walk; the x and y neighbours come from an LDS copy of the plane
// with an R-wide halo (double-buffered: one barrier per plane).  Halo cells
// outside the box hold zeros, which is the Dirichlet condition, so the tap
// loop has no branches.
#include <algorithm>

#include "kernels.h"

namespace tsg {

namespace {

constexpr int kST = 512;  // threads per workgroup

// Conditional load into registers (a value select, so the load stays a
// global load rather than a generic one through a selected pointer).
template <typename T>
__device__ inline void ld_or_zero(const cplx<T>* p, bool ok, T& re, T& im) {
  if (ok) {
    const cplx<T> v = *p;
    re = v.re;
    im = v.im;
  } else {
    re = T(0);
    im = T(0);
  }
}

template <typename T, int R>
__global__ __launch_bounds__(kST) void stencil_kernel(StencilArgs<T> a) {
  extern __shared__ unsigned char smem_raw[];
  cplx<T>* smem = reinterpret_cast<cplx<T>*>(smem_raw);
  const int slot = int(blockIdx.z) / a.ncols, col = int(blockIdx.z) % a.ncols;
  const int w = a.wmap ? a.wmap[slot] : slot;
  if (w < 0) return;  // idle slot (whole workgroup)
  const SysDesc& S = a.sys[a.wsys ? a.wsys[w] : 0];
  const int nx = S.nx, ny = S.ny, nz = S.nz;
  const int tx = a.tx, ty = a.ty;
  const int tilesx = (nx + tx - 1) / tx, tilesy = (ny + ty - 1) / ty;
  if (int(blockIdx.x) >= tilesx * tilesy) return;  // whole workgroup: smaller system
  const int z0 = int(blockIdx.y) * a.zchunk;
  if (z0 >= nz) return;
  const int z1 = min(nz, z0 + a.zchunk);
  const int bx = int(blockIdx.x) % tilesx, by = int(blockIdx.x) / tilesx;
  const int lx = int(threadIdx.x) % tx, ly = int(threadIdx.x) / tx;
  const bool active = ly < ty;
  const int x = bx * tx + lx, y = by * ty + ly;
  const bool inside = active && x < nx && y < ny;
  const int64_t plane = int64_t(nx) * ny;
  const int64_t xy = inside ? int64_t(y) * nx + x : 0;

  const cplx<T>* __restrict__ X = a.X + int64_t(w) * a.wsx + int64_t(col) * a.ldx;
  cplx<T>* __restrict__ Y = a.Y + int64_t(w) * a.wsy + int64_t(col) * a.ldy;
  const T* __restrict__ V;
  const T* __restrict__ G;
  if constexpr (sizeof(T) == 8) { V = reinterpret_cast<const T*>(S.Vd); G = reinterpret_cast<const T*>(S.Gd); }
  else { V = reinterpret_cast<const T*>(S.Vf); G = reinterpret_cast<const T*>(S.Gf); }
  const T diag0 = T(S.diag0);

  const int LW = tx + 2 * R, LH = ty + 2 * R;
  const int nhalo = 2 * R * LW + 2 * R * ty;

  // qr[j], qi[j] hold the value at plane z - R + j (separate real arrays keep
  // the queue in registers)
  T qr[2 * R + 1], qi[2 * R + 1];
#pragma unroll
  for (int j = 0; j < 2 * R + 1; ++j) {
    const int zz = z0 - R + j;
    ld_or_zero(X + zz * plane + xy, inside && zz >= 0 && zz < nz, qr[j], qi[j]);
  }
  for (int z = z0; z < z1; ++z) {
    cplx<T>* L = smem + ((z - z0) & 1) * (LW * LH);
    // the next plane's value is fetched early to overlap its latency
    const int zn = z + R + 1;
    T nr, ni;
    ld_or_zero(X + zn * plane + xy, inside && zn < nz, nr, ni);
    if (active) L[(ly + R) * LW + lx + R] = cplx<T>{qr[R], qi[R]};
    const cplx<T>* __restrict__ Xz = X + z * plane;
    for (int e = int(threadIdx.x); e < nhalo; e += kST) {
      int hx, hy;
      if (e < 2 * R * LW) {  // bands above and below the tile
        hy = e / LW;
        hx = e % LW;
        if (hy >= R) hy += ty;
      } else {               // bands left and right of the tile
        const int f = e - 2 * R * LW;
        hy = R + f / (2 * R);
        const int k = f % (2 * R);
        hx = k < R ? k : tx + k;
      }
      const int gx = bx * tx + hx - R, gy = by * ty + hy - R;
      T hr, hi;
      ld_or_zero(Xz + (int64_t(gy) * nx + gx), gx >= 0 && gx < nx && gy >= 0 && gy < ny, hr, hi);
      L[hy * LW + hx] = cplx<T>{hr, hi};
    }
    __syncthreads();
    if (inside) {
      const int64_t n = z * plane + xy;
      const T d = diag0 + V[n];
      const T g = G[z];
      T ar = d * qr[R] + g * qi[R], ai = d * qi[R] - g * qr[R];
      const cplx<T>* Lc = L + (ly + R) * LW + lx + R;
#pragma unroll
      for (int m = 1; m <= R; ++m) {
        const cplx<T> a = Lc[-m], b = Lc[m], c = Lc[-m * LW], e = Lc[m * LW];
        const T sr = (qr[R - m] + qr[R + m]) + ((a.re + b.re) + (c.re + e.re));
        const T si = (qi[R - m] + qi[R + m]) + ((a.im + b.im) + (c.im + e.im));
        const T cm = T(S.coef[m]);
        ar = fma(cm, sr, ar);
        ai = fma(cm, si, ai);
      }
      Y[n] = cplx<T>{ar, ai};
    }
#pragma unroll
    for (int j = 0; j < 2 * R; ++j) { qr[j] = qr[j + 1]; qi[j] = qi[j + 1]; }
    qr[2 * R] = nr;
    qi[2 * R] = ni;
  }
}

}  // namespace

template <typename T>
void stencil_geometry(StencilArgs<T>& a, int nx, int ny, int nz, int nwin) {
  int tx = 64;
  while (tx > 16 && tx / 2 >= nx) tx /= 2;
  a.tx = tx;
  a.ty = kST / tx;
  a.tiles = ((nx + tx - 1) / tx) * ((ny + a.ty - 1) / a.ty);
  // enough workgroups to fill the chip (a few per compute unit), but z
  // chunks long enough that the 2R planes a chunk re-reads stay minor
  const int64_t base = int64_t(a.tiles) * a.ncols * std::max(nwin, 1);
  int64_t nch = (1024 + base - 1) / base;
  const int minchunk = std::max(32, 4 * a.radius);
  nch = std::max<int64_t>(1, std::min<int64_t>(nch, (nz + minchunk - 1) / minchunk));
  a.zchunk = int((nz + nch - 1) / nch);
}

template <typename T, int R>
void launch_r(const StencilArgs<T>& a, dim3 grid, hipStream_t s) {
  const size_t lds = size_t(2) * (a.tx + 2 * R) * (a.ty + 2 * R) * sizeof(cplx<T>);
  hipLaunchKernelGGL((stencil_kernel<T, R>), grid, dim3(kST), lds, s, a);
}

template <typename T>
void launch_stencil(StencilArgs<T> a, int nwin, int max_nz, hipStream_t s) {
  if (nwin <= 0 || a.ncols <= 0) return;
  dim3 grid(unsigned(a.tiles), unsigned((max_nz + a.zchunk - 1) / a.zchunk), unsigned(nwin * a.ncols));
  switch (a.radius) {
    case 1: launch_r<T, 1>(a, grid, s); break;
    case 2: launch_r<T, 2>(a, grid, s); break;
    case 3: launch_r<T, 3>(a, grid, s); break;
    case 4: launch_r<T, 4>(a, grid, s); break;
    case 5: launch_r<T, 5>(a, grid, s); break;
    default: launch_r<T, 6>(a, grid, s); break;
  }
}

template void launch_stencil<double>(StencilArgs<double>, int, int, hipStream_t);
template void launch_stencil<float>(StencilArgs<float>, int, int, hipStream_t);
template void stencil_geometry<double>(StencilArgs<double>&, int, int, int, int);
template void stencil_geometry<float>(StencilArgs<float>&, int, int, int, int);

}  // namespace tsg
