// H at a Bloch wavevector k on complex FP64 orbitals (interleaved re/im, Nd x Ns column
// major): Sec. 2 of the paper runs every Brillouin-zone sample other than Gamma in complex
// double precision.  Three kernels, launched in this order on one stream:
//   zproject  alpha[v, q] = gamma_q dV sum_{s in S_J} conj(chi~_J[s, a]) x[v, S_J[s]]
//   zhx       out = sa ((T_k + Veff) x - sc x) + sb prev    (Bloch-phased FD ghosts)
//   zscatter  out[v, p] += sa sum_{e in entries of p} chi~[e] alpha[v, col[e]]
// chi~ carries the Bloch phase of the image each support point belongs to (set on the
// host); the three-term filter recurrence uses the same real scalars as the real path.
// Every sum runs in a fixed order: results are bitwise reproducible.
#include "common.h"

namespace chefsi {

namespace {

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 cmulc(double2 a, double2 b) {  // conj(a) * b
  return make_double2(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}

// x~(i + p e_d) for one direction: the wrapped neighbour times the cell phase (periodic),
// or zero outside a Dirichlet boundary.  Periodic directions have n >= r, so i + p wraps
// at most once.
__device__ __forceinline__ double2 neighbour(const double2* __restrict__ xv, int64_t i, int c, int p, int n,
                                             int64_t stride, int periodic, double2 ph) {
  int j = c + p;
  if (j >= n) {
    if (!periodic) return make_double2(0.0, 0.0);
    return cmul(xv[i + (int64_t)(j - n - c) * stride], ph);
  }
  if (j < 0) {
    if (!periodic) return make_double2(0.0, 0.0);
    return cmul(xv[i + (int64_t)(j + n - c) * stride], make_double2(ph.x, -ph.y));
  }
  return xv[i + (int64_t)p * stride];
}

constexpr int kZTx = 32, kZTy = 16;  // plane tile of one block (512 threads)
constexpr int kZLx = kZTx + 2 * kMaxRadius, kZLy = kZTy + 2 * kMaxRadius;

// x~ at (gx, gy) of plane z for any gx, gy within r of the grid: wrapped with the cell
// phases in periodic directions, zero outside a Dirichlet boundary.
__device__ __forceinline__ double2 plane_value(const double2* __restrict__ xv, int gx, int gy, int64_t zoff,
                                               const ZHxArgs& a) {
  double2 f = make_double2(1.0, 0.0);
  const int g[2] = {gx, gy};
  int w[2];
  for (int d = 0; d < 2; ++d) {
    const int n = a.n[d];
    int c = g[d], k = 0;
    while (c >= n) { c -= n; ++k; }
    while (c < 0) { c += n; --k; }
    if (k != 0) {
      if (!a.per[d]) return make_double2(0.0, 0.0);
      const double2 ph = k > 0 ? a.ph[d] : make_double2(a.ph[d].x, -a.ph[d].y);
      for (int t = 0; t < (k > 0 ? k : -k); ++t) f = cmul(f, ph);
    }
    w[d] = c;
  }
  return cmul(xv[zoff + w[0] + (int64_t)a.n[0] * w[1]], f);
}

// One block per (32 x 16 tile of a plane, plane z, orbital): the tile and its r-wide x and y
// halos are staged once in LDS (Bloch phases and Dirichlet zeros applied while staging),
// the x and y neighbours come from LDS, the 2r z neighbours of every point from global
// memory (through the caches).
__global__ __launch_bounds__(kZTx * kZTy) void zhx_kernel(ZHxArgs a) {
  __shared__ double2 tile[kZLy][kZLx];
  const int nx = a.n[0], ny = a.n[1], nz = a.n[2];
  const int tiles_x = (nx + kZTx - 1) / kZTx;
  const int x0 = (blockIdx.x % tiles_x) * kZTx, y0 = (blockIdx.x / tiles_x) * kZTy;
  const int z = blockIdx.y;
  const int64_t v = blockIdx.z;
  const int R = a.r;
  const int64_t pstride = (int64_t)nx * ny;
  const double2* __restrict__ xv = a.x + v * a.nd;
  const int tid = threadIdx.x;
  const int lw = kZTx + 2 * R, lh = kZTy + 2 * R;
  for (int e = tid; e < lw * lh; e += kZTx * kZTy) {
    const int ly = e / lw, lx = e % lw;
    tile[ly][lx] = plane_value(xv, x0 + lx - R, y0 + ly - R, pstride * z, a);
  }
  __syncthreads();
  const int tx = tid % kZTx, ty = tid / kZTx;
  const int x = x0 + tx, y = y0 + ty;
  if (x >= nx || y >= ny) return;
  const int64_t i = x + (int64_t)nx * y + pstride * z;
  const double2 xi = tile[ty + R][tx + R];
  const double diag = a.c0 + a.veff[i] - a.sc;
  double re = diag * xi.x, im = diag * xi.y;
  const double2* col = xv + x + (int64_t)nx * y;
  for (int p = 1; p <= R; ++p) {
    const double2 xu = tile[ty + R][tx + R + p], xd = tile[ty + R][tx + R - p];
    const double2 yu = tile[ty + R + p][tx + R], yd = tile[ty + R - p][tx + R];
    const double2 zu = neighbour(col, pstride * z, z, p, nz, pstride, a.per[2], a.ph[2]);
    const double2 zd = neighbour(col, pstride * z, z, -p, nz, pstride, a.per[2], a.ph[2]);
    re += a.cw[0][p] * (xu.x + xd.x) + a.cw[1][p] * (yu.x + yd.x) + a.cw[2][p] * (zu.x + zd.x);
    im += a.cw[0][p] * (xu.y + xd.y) + a.cw[1][p] * (yu.y + yd.y) + a.cw[2][p] * (zu.y + zd.y);
  }
  double2 o = make_double2(a.sa * re, a.sa * im);
  if (a.prev != nullptr) {
    const double2 pv = a.prev[v * a.nd + i];
    o.x += a.sb * pv.x;
    o.y += a.sb * pv.y;
  }
  a.out[v * a.nd + i] = o;
}

constexpr int kZThreads = 256;

constexpr int kZProj = 4;  // projectors of an atom summed per pass over its support

// one block per (atom, orbital); every thread sums its strided share of the support for
// up to four projectors at once (each support value read once per four projectors), then
// a fixed-shape tree sums the threads
__global__ __launch_bounds__(kZThreads) void zproject_kernel(ZNlArgs a) {
  __shared__ double2 red[kZProj][kZThreads];
  const int J = blockIdx.x;
  const int64_t v = blockIdx.y;
  const int s0 = a.supp_off[J], nj = a.supp_off[J + 1] - s0;
  const int npj = a.nproj[J];
  const int64_t co = a.chi_off[J];
  const double2* __restrict__ xv = a.x + v * a.nd;
  for (int q0 = 0; q0 < npj; q0 += kZProj) {
    const int nq = min(kZProj, npj - q0);
    double2 acc[kZProj];
#pragma unroll
    for (int u = 0; u < kZProj; ++u) acc[u] = make_double2(0.0, 0.0);
    for (int s = threadIdx.x; s < nj; s += kZThreads) {
      const double2 xs = xv[a.supp_idx[s0 + s]];
#pragma unroll
      for (int u = 0; u < kZProj; ++u) {
        if (u < nq) {
          const double2 t = cmulc(a.chi[co + (int64_t)(q0 + u) * nj + s], xs);
          acc[u].x += t.x;
          acc[u].y += t.y;
        }
      }
    }
#pragma unroll
    for (int u = 0; u < kZProj; ++u) red[u][threadIdx.x] = acc[u];
    __syncthreads();
    for (int w = kZThreads / 2; w > 0; w >>= 1) {
      if ((int)threadIdx.x < w) {
#pragma unroll
        for (int u = 0; u < kZProj; ++u) {
          red[u][threadIdx.x].x += red[u][threadIdx.x + w].x;
          red[u][threadIdx.x].y += red[u][threadIdx.x + w].y;
        }
      }
      __syncthreads();
    }
    if ((int)threadIdx.x < nq) {
      const int u = threadIdx.x;
      const int col = a.poff[J] + q0 + u;
      const double g = a.gdv[col];
      a.alpha[v * a.np_tot + col] = make_double2(g * red[u][0].x, g * red[u][0].y);
    }
    __syncthreads();
  }
}

constexpr int kZScatV = 4;  // orbitals per scatter thread (the point's entries read once)

// one thread per (support point, four orbitals); every output element is written by one thread
__global__ __launch_bounds__(256) void zscatter_kernel(ZNsArgs a, int ns) {
  const int p = blockIdx.x * 256 + threadIdx.x;
  if (p >= a.n_pts) return;
  const int64_t v0 = (int64_t)blockIdx.y * kZScatV;
  const int nv = (int)min((int64_t)kZScatV, (int64_t)ns - v0);
  double2 acc[kZScatV];
#pragma unroll
  for (int u = 0; u < kZScatV; ++u) acc[u] = make_double2(0.0, 0.0);
  for (int e = a.ptr[p]; e < a.ptr[p + 1]; ++e) {
    const double2 c = a.val[e];
    const int q = a.col[e];
#pragma unroll
    for (int u = 0; u < kZScatV; ++u) {
      if (u < nv) {
        const double2 t = cmul(c, a.alpha[(v0 + u) * a.np_tot + q]);
        acc[u].x += t.x;
        acc[u].y += t.y;
      }
    }
  }
#pragma unroll
  for (int u = 0; u < kZScatV; ++u) {
    if (u < nv) {
      double2* o = a.out + (v0 + u) * a.nd + a.pt[p];
      double2 cur = *o;
      cur.x += a.sa * acc[u].x;
      cur.y += a.sa * acc[u].y;
      *o = cur;
    }
  }
}

// C(i, j) = sum_q P_q(i, j) for i <= j in a fixed order (P_q column-major ns x ns), then the
// Hermitian completion: C(j, i) = conj(C(i, j)), real diagonal.
__global__ __launch_bounds__(256) void zsum_partials_kernel(const double2* __restrict__ P, int nparts, int ns,
                                                            double2* __restrict__ C) {
  const int64_t n2 = (int64_t)ns * ns;
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= n2) return;
  const int j = (int)(e / ns), i = (int)(e % ns);
  if (i > j) return;
  double re = 0.0, im = 0.0;
  for (int q = 0; q < nparts; ++q) {
    const double2 t = P[q * n2 + e];
    re += t.x;
    im += t.y;
  }
  if (i == j) {
    C[e] = make_double2(re, 0.0);
  } else {
    C[e] = make_double2(re, im);
    C[(int64_t)i * ns + j] = make_double2(re, -im);
  }
}

}  // namespace

hipError_t launch_zsum_partials(const double2* P, int nparts, int ns, double2* C, hipStream_t s) {
  const int64_t n2 = (int64_t)ns * ns;
  hipLaunchKernelGGL(zsum_partials_kernel, dim3((unsigned)((n2 + 255) / 256)), dim3(256), 0, s, P, nparts, ns, C);
  return hipGetLastError();
}

hipError_t launch_zhx(const ZHxArgs& a, int ns, hipStream_t s) {
  if (a.nd <= 0 || ns <= 0) return hipSuccess;
  if (a.r < 1 || a.r > kMaxRadius || a.n[2] > 65535) return hipErrorInvalidValue;
  const int tiles = ((a.n[0] + kZTx - 1) / kZTx) * ((a.n[1] + kZTy - 1) / kZTy);
  dim3 grid((unsigned)tiles, (unsigned)a.n[2], (unsigned)ns);
  hipLaunchKernelGGL(zhx_kernel, grid, dim3(kZTx * kZTy), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_zproject(const ZNlArgs& a, int ns, hipStream_t s) {
  if (a.n_atoms <= 0 || ns <= 0) return hipSuccess;
  hipLaunchKernelGGL(zproject_kernel, dim3((unsigned)a.n_atoms, (unsigned)ns), dim3(kZThreads), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_zscatter(const ZNsArgs& a, int ns, hipStream_t s) {
  if (a.n_pts <= 0 || ns <= 0) return hipSuccess;
  hipLaunchKernelGGL(zscatter_kernel, dim3((unsigned)((a.n_pts + 255) / 256), (unsigned)((ns + kZScatV - 1) / kZScatV)),
                     dim3(256), 0, s, a, ns);
  return hipGetLastError();
}

}  // namespace chefsi
