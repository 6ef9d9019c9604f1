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
#include <string>

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

// YB points per thread, stacked in y (ty = kST / tx thread rows, tile height
// ty * YB): the y taps of a thread's points share one LDS column, and the
// halo per output point shrinks as the tile grows taller.
template <typename T, int R, int YB>
__global__ __launch_bounds__(kST) void stencil_kernel(StencilArgs<T> a) {
  extern __shared__ unsigned char smem_raw[];
  cplx<T>* smem = reinterpret_cast<cplx<T>*>(smem_raw);
  const int slot = int(blockIdx.z) / a.ncols, col = int(blockIdx.z) % a.ncols;
  const int w = a.wmap ? a.wmap[slot] : slot;
  if (w < 0) return;  // idle slot (whole workgroup)
  const SysDesc& S = a.sys[a.wsys ? a.wsys[w] : 0];
  const int nx = S.nx, ny = S.ny, nz = S.nz;
  const int tx = a.tx, ty = a.ty, TY = ty * YB;
  const int tilesx = (nx + tx - 1) / tx, tilesy = (ny + TY - 1) / TY;
  if (int(blockIdx.x) >= tilesx * tilesy) return;  // whole workgroup: smaller system
  const int z0 = int(blockIdx.y) * a.zchunk;
  if (z0 >= nz) return;
  const int z1 = min(nz, z0 + a.zchunk);
  const int bx = int(blockIdx.x) % tilesx, by = int(blockIdx.x) / tilesx;
  const int lx = int(threadIdx.x) % tx, ly = int(threadIdx.x) / tx;
  const bool active = ly < ty;
  const int x = bx * tx + lx, y0 = by * TY + ly * YB;
  const int64_t plane = int64_t(nx) * ny;
  bool inside[YB];
  int64_t xy[YB];
#pragma unroll
  for (int i = 0; i < YB; ++i) {
    inside[i] = active && x < nx && y0 + i < ny;
    xy[i] = inside[i] ? int64_t(y0 + i) * nx + x : 0;
  }

  const cplx<T>* __restrict__ X = a.X + int64_t(w) * a.wsx + int64_t(col) * a.ldx;
  cplx<T>* __restrict__ Y = a.Y + int64_t(w) * a.wsy + int64_t(col) * a.ldy;
  const T* __restrict__ V;
  const T* __restrict__ G;
  if constexpr (sizeof(T) == 8) { V = reinterpret_cast<const T*>(S.Vd); G = reinterpret_cast<const T*>(S.Gd); }
  else { V = reinterpret_cast<const T*>(S.Vf); G = reinterpret_cast<const T*>(S.Gf); }
  const T diag0 = T(S.diag0);

  const int LW = tx + 2 * R, LH = TY + 2 * R;
  const int nhalo = 2 * R * LW + 2 * R * TY;

  // qr[i][j], qi[i][j] hold point i's value at plane z - R + j (separate real
  // arrays keep the queues in registers)
  T qr[YB][2 * R + 1], qi[YB][2 * R + 1];
#pragma unroll
  for (int i = 0; i < YB; ++i)
#pragma unroll
    for (int j = 0; j < 2 * R + 1; ++j) {
      const int zz = z0 - R + j;
      ld_or_zero(X + zz * plane + xy[i], inside[i] && zz >= 0 && zz < nz, qr[i][j], qi[i][j]);
    }
  for (int z = z0; z < z1; ++z) {
    cplx<T>* L = smem + ((z - z0) & 1) * (LW * LH);
    // the next plane's values are fetched early to overlap their latency
    const int zn = z + R + 1;
    T nr[YB], ni[YB];
#pragma unroll
    for (int i = 0; i < YB; ++i) ld_or_zero(X + zn * plane + xy[i], inside[i] && zn < nz, nr[i], ni[i]);
    if (active) {
#pragma unroll
      for (int i = 0; i < YB; ++i) L[(ly * YB + i + R) * LW + lx + R] = cplx<T>{qr[i][R], qi[i][R]};
    }
    const cplx<T>* __restrict__ Xz = X + z * plane;
    for (int e = int(threadIdx.x); e < nhalo; e += kST) {
      int hx, hy;
      if (e < 2 * R * LW) {  // bands above and below the tile
        hy = e / LW;
        hx = e % LW;
        if (hy >= R) hy += TY;
      } else {               // bands left and right of the tile
        const int f = e - 2 * R * LW;
        hy = R + f / (2 * R);
        const int k = f % (2 * R);
        hx = k < R ? k : tx + k;
      }
      const int gx = bx * tx + hx - R, gy = by * TY + hy - R;
      T hr, hi;
      ld_or_zero(Xz + (int64_t(gy) * nx + gx), gx >= 0 && gx < nx && gy >= 0 && gy < ny, hr, hi);
      L[hy * LW + hx] = cplx<T>{hr, hi};
    }
    __syncthreads();
    if (active) {
      const T g = G[z];
      // x taps per point; y taps from one LDS column shared by the YB points
      T ar[YB], ai[YB];
#pragma unroll
      for (int i = 0; i < YB; ++i) {
        const int64_t n = z * plane + xy[i];
        const T d = diag0 + (inside[i] ? V[n] : T(0));
        ar[i] = d * qr[i][R] + g * qi[i][R];
        ai[i] = d * qi[i][R] - g * qr[i][R];
      }
      const cplx<T>* Lc = L + (ly * YB + R) * LW + lx + R;  // point 0
      cplx<T> col[YB + 2 * R];
#pragma unroll
      for (int j = 0; j < YB + 2 * R; ++j) col[j] = Lc[(j - R) * LW];
#pragma unroll
      for (int i = 0; i < YB; ++i) {
        const cplx<T>* Li = Lc + i * LW;
#pragma unroll
        for (int m = 1; m <= R; ++m) {
          const cplx<T> xa = Li[-m], xb = Li[m], c = col[R + i - m], e = col[R + i + m];
          const T sr = (qr[i][R - m] + qr[i][R + m]) + ((xa.re + xb.re) + (c.re + e.re));
          const T si = (qi[i][R - m] + qi[i][R + m]) + ((xa.im + xb.im) + (c.im + e.im));
          const T cm = T(S.coef[m]);
          ar[i] = fma(cm, sr, ar[i]);
          ai[i] = fma(cm, si, ai[i]);
        }
        if (inside[i]) Y[z * plane + xy[i]] = cplx<T>{ar[i], ai[i]};
      }
    }
#pragma unroll
    for (int i = 0; i < YB; ++i) {
#pragma unroll
      for (int j = 0; j < 2 * R; ++j) { qr[i][j] = qr[i][j + 1]; qi[i][j] = qi[i][j + 1]; }
      qr[i][2 * R] = nr[i];
      qi[i][2 * R] = ni[i];
    }
  }
}

}  // namespace

// Tuned geometries, keyed by the largest system's shape, the columns a
// launch covers (window slots x columns) and the element size; filled by
// the autotuner (tune.hip) or from a tuning file.
StencilTuneTable& stencil_tune_table() {
  static StencilTuneTable t;
  return t;
}

template <typename T>
void stencil_geometry(StencilArgs<T>& a, int nx, int ny, int nz, int nwin) {
  StencilGeom gm;
  if (!stencil_tune_table().find(nx, ny, nz, a.ncols * std::max(nwin, 1), int(sizeof(T)), a.radius, gm))
    gm = stencil_default_geometry(nx, ny, nz, a.ncols * std::max(nwin, 1), a.radius);
  stencil_apply_geometry(a, nx, ny, nz, gm);
}

StencilGeom stencil_default_geometry(int nx, int ny, int nz, int64_t launch_cols, int radius) {
  StencilGeom g;
  int tx = 64;
  while (tx > 16 && tx / 2 >= nx) tx /= 2;
  g.tx = tx;
  g.yb = 1;
  const int ty = kST / tx;
  const int64_t tiles = int64_t((nx + tx - 1) / tx) * ((ny + ty - 1) / ty);
  // enough workgroups to fill the chip (a few per compute unit), but z
  // chunks long enough that the 2R planes a chunk re-reads stay minor
  const int64_t base = tiles * std::max<int64_t>(launch_cols, 1);
  int64_t nch = (1024 + base - 1) / base;
  const int minchunk = std::max(32, 4 * radius);
  nch = std::max<int64_t>(1, std::min<int64_t>(nch, (nz + minchunk - 1) / minchunk));
  g.zchunk = int((nz + nch - 1) / nch);
  return g;
}

template <typename T>
void stencil_apply_geometry(StencilArgs<T>& a, int nx, int ny, int nz, const StencilGeom& gm) {
  a.tx = gm.tx;
  a.ty = kST / gm.tx;
  a.yb = gm.yb;
  a.zchunk = std::max(1, std::min(gm.zchunk, nz));
  const int TY = a.ty * a.yb;
  a.tiles = ((nx + a.tx - 1) / a.tx) * ((ny + TY - 1) / TY);
}

template <typename T, int R, int YB>
void launch_r(const StencilArgs<T>& a, dim3 grid, hipStream_t s) {
  const size_t lds = size_t(2) * (a.tx + 2 * R) * (a.ty * YB + 2 * R) * sizeof(cplx<T>);
  if (lds > size_t(64) * 1024) {
    static size_t granted = 0;
    if (lds > granted) {
      const hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(stencil_kernel<T, R, YB>),
                                               hipFuncAttributeMaxDynamicSharedMemorySize, int(lds));
      if (e != hipSuccess) throw DeviceError(std::string("stencil: LDS attribute: ") + hipGetErrorString(e));
      granted = lds;
    }
  }
  hipLaunchKernelGGL((stencil_kernel<T, R, YB>), grid, dim3(kST), lds, s, a);
}

template <typename T, int R>
void launch_yb(const StencilArgs<T>& a, dim3 grid, hipStream_t s) {
  if (a.yb == 2) launch_r<T, R, 2>(a, grid, s);
  else launch_r<T, R, 1>(a, grid, s);
}

template <typename T>
void launch_stencil(StencilArgs<T> a, int nwin, int max_nz, hipStream_t s) {
  if (nwin <= 0 || a.ncols <= 0) return;
  if (a.tx < 1 || kST % a.tx != 0 || (a.yb != 1 && a.yb != 2) || a.zchunk < 1)
    throw DeviceError("stencil: invalid launch geometry");
  dim3 grid(unsigned(a.tiles), unsigned((max_nz + a.zchunk - 1) / a.zchunk), unsigned(nwin * a.ncols));
  switch (a.radius) {
    case 1: launch_yb<T, 1>(a, grid, s); break;
    case 2: launch_yb<T, 2>(a, grid, s); break;
    case 3: launch_yb<T, 3>(a, grid, s); break;
    case 4: launch_yb<T, 4>(a, grid, s); break;
    case 5: launch_yb<T, 5>(a, grid, s); break;
    default: launch_yb<T, 6>(a, grid, s); break;
  }
}

template void launch_stencil<double>(StencilArgs<double>, int, int, hipStream_t);
template void launch_stencil<float>(StencilArgs<float>, int, int, hipStream_t);
template void stencil_geometry<double>(StencilArgs<double>&, int, int, int, int);
template void stencil_geometry<float>(StencilArgs<float>&, int, int, int, int);
template void stencil_apply_geometry<double>(StencilArgs<double>&, int, int, int, const StencilGeom&);
template void stencil_apply_geometry<float>(StencilArgs<float>&, int, int, int, const StencilGeom&);

}  // namespace tsg
