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
// once per walk; the walk is unrolled by 2R+1 planes so that the queue
// advances by renaming registers rather than moving them.  The x and y
// neighbours come from an LDS copy of the plane with an R-wide halo
// (double-buffered: one barrier per plane); each thread's halo cells are
// fixed for the walk, and the next plane's are fetched into registers before
// the barrier.  Halo cells outside the box hold zeros, which is the Dirichlet
// condition, so the tap loop has no branches.
#include <algorithm>
#include <atomic>
#include <string>

#include "kernels.h"

namespace tsg {

namespace {

constexpr int kHaloSlots = 3;  // halo cells per thread and plane, at most
constexpr int kPrefetch = 1;   // planes fetched ahead of the one being computed (measured: 1 is fastest)

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

// NT threads per workgroup (256 or 512).
// YB points per thread, stacked in y (ty = NT / tx thread rows, tile height
// ty * YB): the y taps of a thread's points share one LDS column, and the
// halo per output point shrinks as the tile grows taller.
// CB columns per thread (1 or 2): the columns of a workgroup share its
// barriers, halo offsets, potential and tap weights; each has its own z
// queue and LDS plane.
template <typename T, int R, int YB, int NT, int CB>
__global__ __launch_bounds__(NT) void stencil_kernel(StencilArgs<T> a) {
  extern __shared__ unsigned char smem_raw[];
  cplx<T>* smem = reinterpret_cast<cplx<T>*>(smem_raw);
  // block -> (tile, z chunk, slot and column).  With the XCD-aware order
  // the grid is one-dimensional and padded to a multiple of 8: hardware
  // block b runs on XCD b % 8, and logical block (b % 8) * (nb / 8) + b / 8
  // gives each XCD a contiguous range of logical blocks, tile fastest, so
  // that neighbouring tiles and z chunks (which share halo planes) meet in
  // the same L2.
  int btile, bz, bsc;
  if (a.xcd) {
    const int64_t nb = int64_t(gridDim.x), b = int64_t(blockIdx.x);
    const int64_t L = (b % 8) * (nb / 8) + b / 8;
    if (L >= a.nblocks) return;
    btile = int(L % a.tiles);
    const int64_t rest = L / a.tiles;
    bz = int(rest % a.nzc);
    bsc = int(rest / a.nzc);
  } else {
    btile = int(blockIdx.x);
    bz = int(blockIdx.y);
    bsc = int(blockIdx.z);
  }
  const int ncg = (a.ncols + CB - 1) / CB;  // column groups per window
  const int slot = bsc / ncg, cg = bsc % ncg;
  const int w = a.wmap ? a.wmap[slot] : slot;
  if (w < 0) return;  // idle slot (whole workgroup)
  const SysDesc& S = a.sys[a.wsys ? a.wsys[w] : 0];
  const int nx = S.nx, ny = S.ny, nz = S.nz;
  const int tx = a.tx, ty = a.ty, TY = ty * YB;
  const int tilesx = (nx + tx - 1) / tx, tilesy = (ny + TY - 1) / TY;
  if (btile >= tilesx * tilesy) return;  // whole workgroup: smaller system
  const int z0 = bz * a.zchunk;
  if (z0 >= nz) return;
  const int z1 = min(nz, z0 + a.zchunk);
  const int bx = btile % tilesx, by = btile / tilesx;
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

  // this thread's columns; a missing last column of an odd count reads and
  // writes nothing (its pointers alias the group's first column)
  const cplx<T>* __restrict__ Xc[CB];
  cplx<T>* __restrict__ Yc[CB];
  bool cv[CB];
#pragma unroll
  for (int c = 0; c < CB; ++c) {
    cv[c] = cg * CB + c < a.ncols;
    const int col = cv[c] ? cg * CB + c : cg * CB;
    Xc[c] = a.X + int64_t(w) * a.wsx + int64_t(col) * a.ldx;
    Yc[c] = a.Y + int64_t(w) * a.wsy + int64_t(col) * a.ldy;
  }
  const T* __restrict__ V;
  const T* __restrict__ G;
  if constexpr (sizeof(T) == 8) { V = reinterpret_cast<const T*>(S.Vd); G = reinterpret_cast<const T*>(S.Gd); }
  else { V = reinterpret_cast<const T*>(S.Vf); G = reinterpret_cast<const T*>(S.Gf); }
  const T diag0 = T(S.diag0);

  const int LW = tx + 2 * R, LH = TY + 2 * R;
  const int nhalo = 2 * R * LW + 2 * R * TY;

  // This thread's halo cells, the same for every plane: LDS index (-1: none)
  // and in-plane offset (valid only when the cell lies inside the box; cells
  // outside stay zero, the Dirichlet condition).  kHaloSlots * NT covers the
  // largest halo of the supported geometries (checked at launch).
  int hl[kHaloSlots];
  int64_t hg[kHaloSlots];
  bool hok[kHaloSlots];
#pragma unroll
  for (int k = 0; k < kHaloSlots; ++k) {
    const int e = int(threadIdx.x) + k * NT;
    hl[k] = -1;
    hg[k] = 0;
    hok[k] = false;
    if (e < nhalo) {
      int hx, hy;
      if (e < 2 * R * LW) {  // bands above and below the tile
        hy = e / LW;
        hx = e % LW;
        if (hy >= R) hy += TY;
      } else {               // bands left and right of the tile
        const int f = e - 2 * R * LW;
        hy = R + f / (2 * R);
        const int kk = f % (2 * R);
        hx = kk < R ? kk : tx + kk;
      }
      const int gx = bx * tx + hx - R, gy = by * TY + hy - R;
      hl[k] = hy * LW + hx;
      hok[k] = gx >= 0 && gx < nx && gy >= 0 && gy < ny;
      hg[k] = hok[k] ? int64_t(gy) * nx + gx : 0;
    }
  }

  // z queue and prefetch pipeline.  Planes up to kPrefetch ahead are in
  // flight: at unrolled step s of a group of Q planes (Q >= 2R + kPrefetch, a
  // multiple of kPrefetch), plane z - R + j of point i sits in slot
  // (s + j) % Q, so the queue advances by renaming registers rather than
  // moving them; the halo cells and the potential of plane z sit in ring
  // slot s % kPrefetch.
  T cf[R + 1];  // tap weights, held in registers for the walk
#pragma unroll
  for (int m = 0; m <= R; ++m) cf[m] = T(S.coef[m]);

  constexpr int PD = kPrefetch;
  constexpr int Q = PD * ((2 * R + PD + PD - 1) / PD);
  T qr[CB][YB][Q], qi[CB][YB][Q];
#pragma unroll
  for (int c = 0; c < CB; ++c)
#pragma unroll
    for (int i = 0; i < YB; ++i)
#pragma unroll
      for (int j = 0; j < 2 * R + PD; ++j) {
        const int zz = z0 - R + j;
        ld_or_zero(Xc[c] + zz * plane + xy[i], cv[c] && inside[i] && zz >= 0 && zz < nz, qr[c][i][j], qi[c][i][j]);
      }
  T hr[CB][PD][kHaloSlots], hi[CB][PD][kHaloSlots], vp[PD][YB];
#pragma unroll
  for (int r = 0; r < PD; ++r) {
    const int zz = z0 + r;
#pragma unroll
    for (int c = 0; c < CB; ++c)
#pragma unroll
      for (int k = 0; k < kHaloSlots; ++k)
        ld_or_zero(Xc[c] + zz * plane + hg[k], cv[c] && zz < z1 && hok[k], hr[c][r][k], hi[c][r][k]);
#pragma unroll
    for (int i = 0; i < YB; ++i) vp[r][i] = (zz < z1 && inside[i]) ? V[zz * plane + xy[i]] : T(0);
  }

  for (int zb = z0; zb < z1; zb += Q) {
#pragma unroll
    for (int s = 0; s < Q; ++s) {
      const int z = zb + s;
      if (z >= z1) break;  // uniform over the workgroup
      const int rs = s % PD;
      // column c's plane buffers: CB planes, each double-buffered
      cplx<T>* Lb = smem + ((z - z0) & 1) * (CB * LW * LH);
#pragma unroll
      for (int c = 0; c < CB; ++c) {
        cplx<T>* L = Lb + c * (LW * LH);
        if (active) {
#pragma unroll
          for (int i = 0; i < YB; ++i)
            L[(ly * YB + i + R) * LW + lx + R] = cplx<T>{qr[c][i][(s + R) % Q], qi[c][i][(s + R) % Q]};
        }
#pragma unroll
        for (int k = 0; k < kHaloSlots; ++k)
          if (hl[k] >= 0) L[hl[k]] = cplx<T>{hr[c][rs][k], hi[c][rs][k]};
      }
      T vz[YB];
#pragma unroll
      for (int i = 0; i < YB; ++i) vz[i] = vp[rs][i];
      // plane z + PD's halo and potential and plane z + R + PD's values are
      // fetched before the barrier; their latency overlaps PD planes of taps
      const int zf = z + PD;
      const bool more = zf < z1;
#pragma unroll
      for (int c = 0; c < CB; ++c)
#pragma unroll
        for (int k = 0; k < kHaloSlots; ++k)
          ld_or_zero(Xc[c] + zf * plane + hg[k], cv[c] && more && hok[k], hr[c][rs][k], hi[c][rs][k]);
#pragma unroll
      for (int i = 0; i < YB; ++i) vp[rs][i] = (more && inside[i]) ? V[zf * plane + xy[i]] : T(0);
      const int zn = z + R + PD;
      T nr[CB][YB], ni[CB][YB];
#pragma unroll
      for (int c = 0; c < CB; ++c)
#pragma unroll
        for (int i = 0; i < YB; ++i)
          ld_or_zero(Xc[c] + zn * plane + xy[i], cv[c] && inside[i] && zn < nz, nr[c][i], ni[c][i]);
      __syncthreads();
      if (active) {
        const T g = G[z];
#pragma unroll
        for (int c = 0; c < CB; ++c) {
          const cplx<T>* L = Lb + c * (LW * LH);
          // x taps per point; y taps from one LDS column shared by the YB points
          T ar[YB], ai[YB];
#pragma unroll
          for (int i = 0; i < YB; ++i) {
            const T d = diag0 + vz[i];
            ar[i] = d * qr[c][i][(s + R) % Q] + g * qi[c][i][(s + R) % Q];
            ai[i] = d * qi[c][i][(s + R) % Q] - g * qr[c][i][(s + R) % Q];
          }
          const cplx<T>* Lc = L + (ly * YB + R) * LW + lx + R;  // point 0
          cplx<T> colv[YB + 2 * R];
#pragma unroll
          for (int j = 0; j < YB + 2 * R; ++j) colv[j] = Lc[(j - R) * LW];
#pragma unroll
          for (int i = 0; i < YB; ++i) {
            const cplx<T>* Li = Lc + i * LW;
#pragma unroll
            for (int m = 1; m <= R; ++m) {
              const cplx<T> xa = Li[-m], xb = Li[m], u = colv[R + i - m], e = colv[R + i + m];
              const int lo = (s + R - m) % Q, hi2 = (s + R + m) % Q;
              const T sr = (qr[c][i][lo] + qr[c][i][hi2]) + ((xa.re + xb.re) + (u.re + e.re));
              const T si = (qi[c][i][lo] + qi[c][i][hi2]) + ((xa.im + xb.im) + (u.im + e.im));
              ar[i] = fma(cf[m], sr, ar[i]);
              ai[i] = fma(cf[m], si, ai[i]);
            }
            if (cv[c] && inside[i]) Yc[c][z * plane + xy[i]] = cplx<T>{ar[i], ai[i]};
          }
        }
      }
      // plane z + R + PD enters the queue in the slot after the newest
#pragma unroll
      for (int c = 0; c < CB; ++c)
#pragma unroll
        for (int i = 0; i < YB; ++i) {
          qr[c][i][(s + 2 * R + PD) % Q] = nr[c][i];
          qi[c][i][(s + 2 * R + PD) % Q] = ni[c][i];
        }
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

StencilGeom stencil_lookup(int nx, int ny, int nz, int64_t launch_cols, int elem, int radius, bool* tuned) {
  StencilGeom gm;
  const bool hit = stencil_tune_table().find(nx, ny, nz, launch_cols, elem, radius, gm);
  if (!hit) gm = stencil_default_geometry(nx, ny, nz, launch_cols, radius);
  if (tuned) *tuned = hit;
  return gm;
}

template <typename T>
void stencil_geometry(StencilArgs<T>& a, int nx, int ny, int nz, int nwin) {
  // keyed by the complex element size, as the autotuner records it
  const StencilGeom gm = stencil_lookup(nx, ny, nz, int64_t(a.ncols) * std::max(nwin, 1), int(sizeof(cplx<T>)),
                                        a.radius, nullptr);
  stencil_apply_geometry(a, nx, ny, nz, gm);
}

bool stencil_geometry_valid(const StencilGeom& g, int radius, int elem) {
  if (g.nt != 256 && g.nt != 512) return false;
  // two columns per thread only for complex64 (complex128 would spill)
  if (g.cb != 1 && !(g.cb == 2 && elem == 8)) return false;
  if (g.tx < 1 || g.nt % g.tx != 0 || (g.yb != 1 && g.yb != 2) || g.zchunk < 1 || (g.xcd != 0 && g.xcd != 1))
    return false;
  if (radius < 1 || radius > 6) return false;
  const int64_t TY = int64_t(g.nt / g.tx) * g.yb;
  const int64_t nhalo = 2 * int64_t(radius) * (g.tx + 2 * radius) + 2 * int64_t(radius) * TY;
  return nhalo <= int64_t(kHaloSlots) * g.nt;  // each thread holds at most kHaloSlots halo cells
}

StencilGeom stencil_default_geometry(int nx, int ny, int nz, int64_t launch_cols, int radius) {
  StencilGeom g;
  int tx = 64;
  while (tx > 16 && tx / 2 >= nx) tx /= 2;
  g.tx = tx;
  g.yb = 1;
  g.nt = 512;
  const int ty = g.nt / tx;
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
  a.nt = gm.nt;
  a.cb = gm.cb;
  a.ty = gm.tx > 0 ? gm.nt / gm.tx : 0;
  a.yb = gm.yb;
  a.xcd = gm.xcd;
  a.zchunk = std::max(1, std::min(gm.zchunk, nz));
  const int TY = a.ty * a.yb;
  a.tiles = ((nx + a.tx - 1) / a.tx) * ((ny + TY - 1) / TY);
}

template <typename T, int R, int YB, int NT, int CB>
void launch_r(const StencilArgs<T>& a, dim3 grid, hipStream_t s) {
  const size_t lds = size_t(2) * CB * (a.tx + 2 * R) * (a.ty * YB + 2 * R) * sizeof(cplx<T>);
  if (lds > size_t(64) * 1024) {
    static std::atomic<size_t> granted{0};
    if (lds > granted.load()) {
      const hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(stencil_kernel<T, R, YB, NT, CB>),
                                               hipFuncAttributeMaxDynamicSharedMemorySize, int(lds));
      if (e != hipSuccess) throw DeviceError(std::string("stencil: LDS attribute: ") + hipGetErrorString(e));
      size_t cur = granted.load();
      while (lds > cur && !granted.compare_exchange_weak(cur, lds)) {
      }
    }
  }
  hipLaunchKernelGGL((stencil_kernel<T, R, YB, NT, CB>), grid, dim3(NT), lds, s, a);
}

template <typename T, int R, int NT, int CB>
void launch_y(const StencilArgs<T>& a, dim3 grid, hipStream_t s) {
  if (a.yb == 2) launch_r<T, R, 2, NT, CB>(a, grid, s);
  else launch_r<T, R, 1, NT, CB>(a, grid, s);
}

template <typename T, int R>
void launch_yb(const StencilArgs<T>& a, dim3 grid, hipStream_t s) {
  if constexpr (sizeof(T) == 4) {
    if (a.cb == 2) {
      if (a.nt == 256) launch_y<T, R, 256, 2>(a, grid, s);
      else launch_y<T, R, 512, 2>(a, grid, s);
      return;
    }
  }
  if (a.nt == 256) launch_y<T, R, 256, 1>(a, grid, s);
  else launch_y<T, R, 512, 1>(a, grid, s);
}

template <typename T>
void launch_stencil(StencilArgs<T> a, int nwin, int max_nz, hipStream_t s) {
  if (nwin <= 0 || a.ncols <= 0) return;
  if (!stencil_geometry_valid(StencilGeom{a.tx, a.yb, a.zchunk, a.xcd, a.nt, a.cb}, a.radius,
                              int(sizeof(cplx<T>))))
    throw DeviceError("stencil: invalid launch geometry");
  a.nzc = (max_nz + a.zchunk - 1) / a.zchunk;
  const int ncg = (a.ncols + a.cb - 1) / a.cb;
  a.nblocks = int64_t(a.tiles) * a.nzc * nwin * ncg;
  dim3 grid(unsigned(a.tiles), unsigned(a.nzc), unsigned(nwin * ncg));
  if (a.xcd) {
    const int64_t padded = ((a.nblocks + 7) / 8) * 8;
    // the dispatch counts work-items in 32 bits
    if (padded * a.nt > int64_t(0xffffffff)) throw DeviceError("stencil: grid too large for the XCD-aware order");
    grid = dim3(unsigned(padded), 1, 1);
  }
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
