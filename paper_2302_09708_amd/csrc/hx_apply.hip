// hx_apply: matrix-free Kohn-Sham H on a block of orbitals, fused with the Chebyshev update.
//
// Sec. 2.1 applies H in three parts: the finite-difference Laplacian stencil of
// order n0 = 2r (3 n0 + 1 operations per output point), the pointwise Veff
// product and the Kleinman-Bylander projectors.  Here the three are one pass
// over HBM, and the Chebyshev three-term update of Alg. 1 (scaled form) is the
// epilogue, so one launch reads Y_k and Y_{k-1} once and writes Y_{k+1} once:
//
//   out[i] = sa * ((H y)[i] - sc * y[i]) + sb * prev[i]
//
// Mapping on gfx950 (wave64, 160 KB LDS per CU):
//   * one block = one orbital x one tile of whole x-rows (nx wide, ty = nyg*PY
//     rows) x one chunk of z-planes; a thread owns PY consecutive y rows at one x;
//   * the block marches through z.  Each thread keeps its 2r+1 z-neighbours in a
//     register queue (the z part of the stencil never touches LDS) and prefetches
//     the next plane one iteration ahead;
//   * the current plane of the tile plus r halo rows above and below sits in LDS;
//     x neighbours wrap inside the row (periodic) or read as zero (Dirichlet), so
//     whole-row tiles need no x halo at all; y neighbours are read once per
//     column and reused by the PY rows the thread owns;
//   * the projector term is gathered from a point-major table (no atomics, fixed
//     summation order, so results are bitwise reproducible).
#include "common.h"

#include <algorithm>
#include <cstdlib>

namespace chefsi {

__device__ __forceinline__ int wrap_index(int v, int n) {
  v %= n;
  return v < 0 ? v + n : v;
}

// Offset of row gy inside a plane (x added), or -1 for a Dirichlet zero row.
__device__ __forceinline__ int row_offset(int x, int gy, int nx, int ny, int per_y) {
  if (per_y) return x + nx * wrap_index(gy, ny);
  return (gy < 0 || gy >= ny) ? -1 : x + nx * gy;
}

// Offset of plane pz, or -1 for a Dirichlet zero plane.
__device__ __forceinline__ int plane_offset(int pz, int nplane, int nz, int per_z) {
  if (per_z) return nplane * wrap_index(pz, nz);
  return (pz < 0 || pz >= nz) ? -1 : nplane * pz;
}

template <typename TI>
__device__ __forceinline__ TI load_at(const TI* __restrict__ xv, int roff, int poff) {
  return (roff < 0 || poff < 0) ? TI(0) : xv[roff + poff];
}

template <typename TI, typename TC, typename TO, int R, int PY>
__global__ __launch_bounds__(512) void hx_apply_kernel(HxArgs<TI, TC, TO> a) {
  extern __shared__ __align__(16) unsigned char lds_raw[];
  TI* lds = reinterpret_cast<TI*>(lds_raw);

  constexpr int Q = 2 * R + 1;
  constexpr int kMaxHalo = kHxMaxHalo;  // halo values per thread (planner keeps 2R*nx <= kMaxHalo*blockDim)
  const int nx = a.nx, ny = a.ny, nz = a.nz;
  const int tid = threadIdx.x;
  const int nthr = blockDim.x;
  const int used = nx * a.nyg;
  const bool active = tid < used;
  const int x = active ? tid % nx : 0;
  const int yg = active ? tid / nx : 0;
  const int tile = blockIdx.x % a.nty;
  const int zchunk = blockIdx.x / a.nty;
  const int64_t vec = blockIdx.y;
  const int y0 = tile * a.ty;
  const int z0 = zchunk * a.zc;
  const int z1 = min(z0 + a.zc, nz);
  if (z0 >= nz) return;

  const TI* __restrict__ xv = a.x + vec * a.nd;
  const int ly0 = yg * PY;  // first local row of this thread

  const int nplane = nx * ny;
  int roff[PY];
#pragma unroll
  for (int j = 0; j < PY; ++j) roff[j] = active ? row_offset(x, y0 + ly0 + j, nx, ny, a.per_y) : -1;

  // register queue: q[s][j] = value at plane (z - R + s), row y0 + ly0 + j
  TI q[Q][PY];
  TI pf[PY];
#pragma unroll
  for (int j = 0; j < PY; ++j) q[0][j] = TI(0);
#pragma unroll
  for (int s = 1; s < Q; ++s) {
    const int po = plane_offset(z0 - R - 1 + s, nplane, nz, a.per_z);
#pragma unroll
    for (int j = 0; j < PY; ++j) q[s][j] = load_at(xv, roff[j], po);
  }
  {
    const int po = plane_offset(z0 + R, nplane, nz, a.per_z);
#pragma unroll
    for (int j = 0; j < PY; ++j) pf[j] = load_at(xv, roff[j], po);
  }

  // halo rows: local LDS rows [0, R) and [R + ty, ty + 2R), i.e. global rows y0 - R + yy
  const int nhalo = 2 * R * nx;
  const int kh = (nhalo + nthr - 1) / nthr;
  TI hpf[kMaxHalo];
  int hoff[kMaxHalo];   // source offset inside a plane (-1: zero row or unused slot)
  int hdst[kMaxHalo];   // destination in LDS
  {
    const int po = plane_offset(z0, nplane, nz, a.per_z);
#pragma unroll
    for (int k = 0; k < kMaxHalo; ++k) {
      const int e = tid + k * nthr;
      hoff[k] = -1;
      hdst[k] = -1;
      if (k < kh && e < nhalo) {
        const int hr = e / nx, hxx = e % nx;
        const int yy = hr < R ? hr : hr + a.ty;
        hoff[k] = row_offset(hxx, y0 - R + yy, nx, ny, a.per_y);
        hdst[k] = yy * nx + hxx;
      }
      hpf[k] = load_at(xv, hoff[k], po);
    }
  }

  const int row_stride = nx;
  for (int z = z0; z < z1; ++z) {
    // advance the queue; the plane z + R arrived in pf during the previous iteration
#pragma unroll
    for (int s = 0; s < Q - 1; ++s)
#pragma unroll
      for (int j = 0; j < PY; ++j) q[s][j] = q[s + 1][j];
#pragma unroll
    for (int j = 0; j < PY; ++j) q[Q - 1][j] = pf[j];
    if (z + 1 < z1) {
      const int po = plane_offset(z + 1 + R, nplane, nz, a.per_z);
#pragma unroll
      for (int j = 0; j < PY; ++j) pf[j] = load_at(xv, roff[j], po);
    }

    // epilogue operands for this plane, issued early
    TC vpot[PY], vprev[PY];
    int64_t gidx[PY];
    bool valid[PY];
#pragma unroll
    for (int j = 0; j < PY; ++j) {
      const int gy = y0 + ly0 + j;
      valid[j] = active && gy < ny;
      gidx[j] = valid[j] ? (int64_t)(x + nx * gy + nplane * z) : 0;
      vpot[j] = valid[j] ? a.veff[gidx[j]] : TC(0);
      vprev[j] = (valid[j] && a.prev != nullptr) ? TC(a.prev[vec * a.nd + gidx[j]]) : TC(0);
    }

    __syncthreads();  // previous plane's LDS reads are done
    if (active) {
#pragma unroll
      for (int j = 0; j < PY; ++j) lds[(R + ly0 + j) * row_stride + x] = q[R][j];
    }
    {
      const int po = (z + 1 < z1) ? plane_offset(z + 1, nplane, nz, a.per_z) : -1;
#pragma unroll
      for (int k = 0; k < kMaxHalo; ++k) {
        if (hdst[k] >= 0) {
          lds[hdst[k]] = hpf[k];
          hpf[k] = load_at(xv, hoff[k], po);
        }
      }
    }
    __syncthreads();

    if (active) {
      TC acc[PY];
#pragma unroll
      for (int j = 0; j < PY; ++j) {
        const TC v = TC(q[R][j]);
        TC t = a.c0 * v;
#pragma unroll
        for (int p = 1; p <= R; ++p) t += a.cz[p] * (TC(q[R + p][j]) + TC(q[R - p][j]));
        acc[j] = t;
      }
      // y part: one read per LDS row of the column, shared by the PY outputs
      TC col[PY + 2 * R];
#pragma unroll
      for (int t = 0; t < PY + 2 * R; ++t) col[t] = TC(lds[(ly0 + t) * row_stride + x]);
#pragma unroll
      for (int j = 0; j < PY; ++j)
#pragma unroll
        for (int p = 1; p <= R; ++p) acc[j] += a.cy[p] * (col[R + j + p] + col[R + j - p]);
      // x part: neighbours inside the row
#pragma unroll
      for (int j = 0; j < PY; ++j) {
        const TI* row = lds + (R + ly0 + j) * row_stride;
        TC t = TC(0);
        if (a.per_x) {
#pragma unroll
          for (int p = 1; p <= R; ++p) {
            int xp = x + p;
            xp = xp >= nx ? xp - nx : xp;
            int xm = x - p;
            xm = xm < 0 ? xm + nx : xm;
            t += a.cx[p] * (TC(row[xp]) + TC(row[xm]));
          }
        } else {
#pragma unroll
          for (int p = 1; p <= R; ++p) {
            const TC vp = (x + p < nx) ? TC(row[x + p]) : TC(0);
            const TC vm = (x - p >= 0) ? TC(row[x - p]) : TC(0);
            t += a.cx[p] * (vp + vm);
          }
        }
        acc[j] += t;
      }
#pragma unroll
      for (int j = 0; j < PY; ++j) {
        if (!valid[j]) continue;
        const TC v = TC(q[R][j]);
        TC hy = acc[j] + vpot[j] * v;
        if (a.nl_row != nullptr) {
          const int e0 = a.nl_row[gidx[j]], e1 = a.nl_row[gidx[j] + 1];
          TC nl = TC(0);
          const TC* al = a.alpha + vec * a.np_tot;
          for (int e = e0; e < e1; ++e) nl += a.nl_val[e] * al[a.nl_proj[e]];
          hy += nl;
        }
        TC r = a.sa * (hy - a.sc * v);
        if (a.prev != nullptr) r += a.sb * vprev[j];
        a.out[vec * a.nd + gidx[j]] = TO(r);
      }
    }
  }
}

HxPlan plan_hx(int nx, int ny, int nz, int ns, int radius, int elem_bytes, int py_override) {
  HxPlan best;
  double best_cost = 1e300;
  const int pys[] = {1, 2, 3, 4};
  for (int py : pys) {
    if (py_override > 0 && py != py_override) continue;
    if (py_override <= 0 && elem_bytes == 8 && py > 2) continue;  // FP64 register queue budget
    for (int nyg = 1; nx * nyg <= kHxMaxThreads; ++nyg) {
      const int ty = nyg * py;
      const int nty = (ny + ty - 1) / ty;
      const int threads = nx * nyg;
      const int waves = (threads + 63) / 64;
      if (2 * radius * nx > kHxMaxHalo * waves * 64) continue;  // halo values per thread bound
      const size_t lds = (size_t)(ty + 2 * radius) * nx * elem_bytes;
      if (lds > 64 * 1024) continue;
      const double lane_eff = (double)threads / (waves * 64.0);
      const double row_eff = (double)ny / (nty * ty);
      const double halo = (double)(ty + 2 * radius) / ty;
      double cost = 1.0 / (lane_eff * row_eff) * (1.0 + 0.35 * (halo - 1.0));
      if (threads < 128) cost *= 1.15;
      if (ty > ny + 2 * radius) cost *= 2.0;
      if (cost < best_cost - 1e-12) {
        best_cost = cost;
        best.ok = true;
        best.py = py;
        best.nyg = nyg;
        best.ty = ty;
        best.nty = nty;
        best.threads = waves * 64;
        best.lds_bytes = lds;
      }
    }
  }
  // z chunks: enough blocks to fill 256 CUs several times over, chunks no thinner than 2r planes
  const int64_t xyblocks = (int64_t)best.nty * ns;
  int nzc = (int)std::max<int64_t>(1, (2048 + xyblocks - 1) / xyblocks);
  nzc = std::min(nzc, std::max(1, nz / std::max(1, 2 * radius)));
  best.zc = (nz + nzc - 1) / nzc;
  best.nzc = (nz + best.zc - 1) / best.zc;
  return best;
}

template <typename TI, typename TC, typename TO, int R, int PY>
static hipError_t launch_rp(const HxArgs<TI, TC, TO>& a, const HxPlan& p, int ns, hipStream_t s) {
  dim3 grid((unsigned)(p.nty * p.nzc), (unsigned)ns);
  hipLaunchKernelGGL((hx_apply_kernel<TI, TC, TO, R, PY>), grid, dim3(p.threads), p.lds_bytes, s, a);
  return hipGetLastError();
}

template <typename TI, typename TC, typename TO, int R>
static hipError_t launch_r(const HxArgs<TI, TC, TO>& a, const HxPlan& p, int ns, hipStream_t s) {
  switch (p.py) {
    case 1: return launch_rp<TI, TC, TO, R, 1>(a, p, ns, s);
    case 2: return launch_rp<TI, TC, TO, R, 2>(a, p, ns, s);
    case 3: return launch_rp<TI, TC, TO, R, 3>(a, p, ns, s);
    case 4: return launch_rp<TI, TC, TO, R, 4>(a, p, ns, s);
    default: return hipErrorInvalidValue;
  }
}

template <typename TI, typename TC, typename TO>
hipError_t launch_hx(const HxArgs<TI, TC, TO>& a, const HxPlan& p, int radius, int ns, hipStream_t s) {
  if (ns <= 0) return hipSuccess;
  if (!p.ok) return hipErrorInvalidConfiguration;
  switch (radius) {
    case 1: return launch_r<TI, TC, TO, 1>(a, p, ns, s);
    case 2: return launch_r<TI, TC, TO, 2>(a, p, ns, s);
    case 3: return launch_r<TI, TC, TO, 3>(a, p, ns, s);
    case 4: return launch_r<TI, TC, TO, 4>(a, p, ns, s);
    case 5: return launch_r<TI, TC, TO, 5>(a, p, ns, s);
    case 6: return launch_r<TI, TC, TO, 6>(a, p, ns, s);
    default: return hipErrorInvalidValue;
  }
}

template hipError_t launch_hx<double, double, double>(const HxArgs<double, double, double>&, const HxPlan&, int, int,
                                                      hipStream_t);
template hipError_t launch_hx<float, float, float>(const HxArgs<float, float, float>&, const HxPlan&, int, int,
                                                   hipStream_t);
template hipError_t launch_hx<float, double, double>(const HxArgs<float, double, double>&, const HxPlan&, int, int,
                                                     hipStream_t);

}  // namespace chefsi
