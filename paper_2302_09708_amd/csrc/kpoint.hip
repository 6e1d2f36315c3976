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

#include <algorithm>

namespace chefsi {

namespace {

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 cmulc(double2 a, double2 b) {  // conj(a) * b
  return make_double2(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}

// ---------------------------------------------------------------------------
// zhx: the Bloch-phased stencil pass, laid out like the real one.  One block = one orbital
// x a tile of whole x rows (ty rows, one row per thread) x a chunk of z planes; the block
// marches through z with the 2r+1 z neighbours of its column in registers, and stages each
// plane of the tile plus r halo rows (and r periodic copies on each side of every row) in
// double-buffered LDS.  Every value that crosses a periodic face carries the cell phase
// exp(+-i k_d L_d) of that face: the staged slots keep their phase (a constant per slot),
// the z queue multiplies the plane's phase into its loads, and rows past ny of the last
// tile (periodic y) carry exp(i k_y L_y).  Zero ghosts of Dirichlet faces are buffer loads
// past the end of the resource (no branch).
// ---------------------------------------------------------------------------
constexpr unsigned kZOOB = 0x80000000u;
constexpr int kZDummy = 64;  // per-lane dummy LDS slots after each buffer

__device__ __forceinline__ __amdgpu_buffer_rsrc_t zrsrc(const void* p, int64_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, (int)bytes, 0x00020000);
}
__device__ __forceinline__ double2 zload(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff) {
  const auto v = __builtin_amdgcn_raw_buffer_load_b128(r, voff, soff, 0);
  const unsigned v0 = v[0], v1 = v[1], v2 = v[2], v3 = v[3];
  return make_double2(__builtin_bit_cast(double, (unsigned long long)v0 | ((unsigned long long)v1 << 32)),
                      __builtin_bit_cast(double, (unsigned long long)v2 | ((unsigned long long)v3 << 32)));
}
__device__ __forceinline__ void zstore(__amdgpu_buffer_rsrc_t r, double2 v, unsigned voff, unsigned soff) {
  typedef unsigned u32x4z __attribute__((__vector_size__(16)));
  const unsigned long long a = __builtin_bit_cast(unsigned long long, v.x);
  const unsigned long long b = __builtin_bit_cast(unsigned long long, v.y);
  u32x4z w = {(unsigned)a, (unsigned)(a >> 32), (unsigned)b, (unsigned)(b >> 32)};
  __builtin_amdgcn_raw_buffer_store_b128(w, r, voff, soff, 0);
}
__device__ __forceinline__ unsigned zoff(int e) { return e < 0 ? kZOOB : (unsigned)e * 16u; }
__device__ __forceinline__ double2 zpow(double2 ph, int k) {  // ph^k, k of either sign
  double2 f = make_double2(1.0, 0.0);
  const double2 b = k >= 0 ? ph : make_double2(ph.x, -ph.y);
  for (int t = 0; t < (k >= 0 ? k : -k); ++t) f = cmul(f, b);
  return f;
}
// wrap c into [0, n): the wrapped index and the number of cells crossed (k)
__device__ __forceinline__ int zwrap(int c, int n, int& k) {
  k = 0;
  while (c >= n) { c -= n; ++k; }
  while (c < 0) { c += n; --k; }
  return c;
}

template <int R, int KH>
__global__ __launch_bounds__(kZMaxThreads) void zhx_kernel(ZHxArgs a, ZTiling t) {
  extern __shared__ __align__(16) unsigned char zlds[];
  constexpr int Q = 2 * R + 1;
  const int nx = a.n[0], ny = a.n[1], nz = a.n[2];
  const int tid = threadIdx.x, nthr = blockDim.x, lane = tid & 63;
  const int64_t logical = (int64_t)(blockIdx.x % 8) * t.per_xcd + blockIdx.x / 8;
  if (logical >= t.nblocks) return;
  const int per_vec = t.nty * t.nzc;
  const int64_t vec = logical / per_vec;
  const int rem = (int)(logical % per_vec);
  const int y0 = (rem % t.nty) * t.ty, z0 = (rem / t.nty) * t.zc;
  const int z1 = min(z0 + t.zc, nz);
  const int nzl = z1 - z0;
  const int pitch = t.pitch;
  const int tile_elems = (t.ty + 2 * R) * pitch, tile_buf = tile_elems + kZDummy;
  double2* lt = reinterpret_cast<double2*>(zlds);

  const int nplane = nx * ny;
  const int xbytes = (int)(a.nd * 16);
  const __amdgpu_buffer_rsrc_t rx = zrsrc(a.x + vec * a.nd, xbytes);
  const __amdgpu_buffer_rsrc_t rzero = zrsrc(a.x, 0);
  const __amdgpu_buffer_rsrc_t rv = zrsrc(a.veff, a.nd * 8);
  const bool has_prev = a.prev != nullptr;
  const __amdgpu_buffer_rsrc_t rp = zrsrc(has_prev ? (const void*)(a.prev + vec * a.nd) : (const void*)a.out,
                                          has_prev ? xbytes : 0);
  const __amdgpu_buffer_rsrc_t ro = zrsrc(a.out + vec * a.nd, xbytes);

  // the thread's row: offset in a plane (kZOOB for a Dirichlet zero row), the phase of a
  // wrapped row, whether its output is stored, and its LDS slot (a dummy for idle lanes)
  const bool active = tid < nx * t.ty;
  const int x = active ? tid % nx : 0, ly = active ? tid / nx : 0;
  const int gy = y0 + ly;
  int ky;
  const int wy = zwrap(gy, ny, ky);
  const bool rowzero = !active || (ky != 0 && !a.per[1]);
  const unsigned vq = rowzero ? kZOOB : (unsigned)(x + nx * wy) * 16u;
  const double2 rowph = zpow(a.ph[1], ky);
  const bool valid = active && gy < ny;
  const unsigned vo = valid ? (unsigned)(x + nx * gy) * 16u : kZOOB;
  const unsigned vv = valid ? (unsigned)(x + nx * gy) * 8u : kZOOB;
  const int sown = active ? (R + ly) * pitch + R + x : tile_elems + lane;

  // staged slots: halo rows (and, with a periodic x, the r copies on each side of every row)
  int sdst[KH];
  unsigned vh[KH];
  double2 sph[KH];
  {
    const int w = a.per[0] ? nx + 2 * R : nx;
    const int nslots = 2 * R * w + (a.per[0] ? t.ty * 2 * R : 0);
#pragma unroll
    for (int k = 0; k < KH; ++k) {
      const int e = tid + k * nthr;
      sdst[k] = tile_elems + lane;
      vh[k] = kZOOB;
      sph[k] = make_double2(1.0, 0.0);
      if (e < nslots) {
        int yy, c;
        if (e < 2 * R * w) {
          const int hr = e / w;
          c = e % w + (a.per[0] ? 0 : R);
          yy = hr < R ? hr : hr + t.ty;
        } else {
          const int f = e - 2 * R * w;
          const int cc = f % (2 * R);
          c = cc < R ? cc : nx + cc;
          yy = R + f / (2 * R);
        }
        int kx, kyy;
        const int sx = zwrap(c - R, nx, kx);
        const int sy = zwrap(y0 - R + yy, ny, kyy);
        sdst[k] = yy * pitch + c;
        const bool zero = (kx != 0 && !a.per[0]) || (kyy != 0 && !a.per[1]);
        vh[k] = zero ? kZOOB : (unsigned)(sx + nx * sy) * 16u;
        sph[k] = cmul(zpow(a.ph[0], kx), zpow(a.ph[1], kyy));
      }
    }
  }

  // plane p of the z queue: the wrapped plane's byte offset and resource, and its phase
  auto qplane = [&](int p, __amdgpu_buffer_rsrc_t& r, unsigned& so, double2& ph) {
    int kz;
    const int wz = zwrap(p, nz, kz);
    const bool zero = kz != 0 && !a.per[2];
    r = zero ? rzero : rx;
    so = zero ? 0u : (unsigned)wz * (unsigned)nplane * 16u;
    ph = cmul(zpow(a.ph[2], kz), rowph);
  };

  double2 q[Q], pf, hp[KH];
  q[0] = make_double2(0.0, 0.0);
#pragma unroll
  for (int s = 1; s < Q; ++s) {
    __amdgpu_buffer_rsrc_t r;
    unsigned so;
    double2 ph;
    qplane(z0 - R - 1 + s, r, so, ph);
    q[s] = cmul(zload(r, vq, so), ph);
  }
  __amdgpu_buffer_rsrc_t rpf;
  unsigned spf;
  double2 phf;
  qplane(z0 + R, rpf, spf, phf);
  pf = zload(rpf, vq, spf);
#pragma unroll
  for (int k = 0; k < KH; ++k) hp[k] = zload(rx, vh[k], (unsigned)z0 * (unsigned)nplane * 16u);

  if (!a.per[0]) {  // Dirichlet x: the halo columns of both buffers hold zeros
    const int rows = 2 * (t.ty + 2 * R);
    for (int i = tid; i < rows * 2 * R; i += nthr) {
      const int row = i / (2 * R), c = i % (2 * R);
      const int buf = row / (t.ty + 2 * R), rr = row % (t.ty + 2 * R);
      lt[buf * tile_buf + rr * pitch + (c < R ? c : nx + c)] = make_double2(0.0, 0.0);
    }
  }

  for (int zl = 0; zl < nzl; ++zl) {
    const int z = z0 + zl;
    double2* tl = lt + (zl & 1) * tile_buf;
    const bool more = zl + 1 < nzl;
    const unsigned zo = (unsigned)z * (unsigned)nplane;
    const double vz = __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(rv, vv, zo * 8u, 0));
    const double2 cp = zload(rp, vo, zo * 16u);
    // advance the queue (the fetched plane's phase applied now); fetch plane z + R + 1
#pragma unroll
    for (int s = 0; s < Q - 1; ++s) q[s] = q[s + 1];
    q[Q - 1] = cmul(pf, phf);
    if (more) qplane(z + R + 1, rpf, spf, phf);
    else {
      rpf = rzero;
      spf = 0u;
    }
    pf = zload(rpf, vq, spf);
    // stage plane z; fetch the staged values of plane z + 1
    tl[sown] = q[R];
#pragma unroll
    for (int k = 0; k < KH; ++k) tl[sdst[k]] = cmul(hp[k], sph[k]);
    {
      const __amdgpu_buffer_rsrc_t r = more ? rx : rzero;
      const unsigned so = more ? (unsigned)(z + 1) * (unsigned)nplane * 16u : 0u;
#pragma unroll
      for (int k = 0; k < KH; ++k) hp[k] = zload(r, vh[k], so);
    }
    __syncthreads();

    const double2 xc = q[R];
    const double dg = a.c0 + vz - a.sc;
    double re = dg * xc.x, im = dg * xc.y;
    const double2* row = tl + (R + ly) * pitch + R + x;
#pragma unroll
    for (int p = 1; p <= R; ++p) {
      const double2 xu = row[p], xd = row[-p];
      const double2 yu = row[p * pitch], yd = row[-p * pitch];
      const double2 zu = q[R + p], zd = q[R - p];
      re += a.cw[0][p] * (xu.x + xd.x) + a.cw[1][p] * (yu.x + yd.x) + a.cw[2][p] * (zu.x + zd.x);
      im += a.cw[0][p] * (xu.y + xd.y) + a.cw[1][p] * (yu.y + yd.y) + a.cw[2][p] * (zu.y + zd.y);
    }
    zstore(ro, make_double2(a.sa * re + a.sb * cp.x, a.sa * im + a.sb * cp.y), vo, zo * 16u);
  }
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

ZTiling plan_zhx(int nx, int ny, int nz, int ns, int radius) {
  ZTiling t{};
  // rows per tile: whole x rows, one per thread, at most kZMaxThreads threads; at least
  // r + 1 rows when they fit (thinner tiles read the halo more than twice per row)
  t.ty = std::max(1, std::min(ny, kZMaxThreads / std::max(1, nx)));
  t.nty = (ny + t.ty - 1) / t.ty;
  t.threads = ((nx * t.ty + 63) / 64) * 64;
  t.pitch = nx + std::max(16, ((2 * radius + 15) / 16) * 16);  // row gap of 256 bytes: distinct banks
  const int w = nx + 2 * radius;
  const int nslots = 2 * radius * w + t.ty * 2 * radius;
  t.kh = std::max(2, (nslots + t.threads - 1) / t.threads);
  const int64_t xy = (int64_t)t.nty * ns;
  int nzc = (int)std::max<int64_t>(1, (2048 + xy - 1) / xy);
  nzc = std::min(nzc, std::max(1, nz / std::max(1, 2 * radius)));
  t.zc = (nz + nzc - 1) / nzc;
  t.nzc = (nz + t.zc - 1) / t.zc;
  t.lds_bytes = 2 * ((size_t)(t.ty + 2 * radius) * t.pitch + kZDummy) * 16;
  return t;
}

template <int R>
static hipError_t launch_zhx_r(const ZHxArgs& a, ZTiling t, int ns, hipStream_t s) {
  t.nblocks = (int64_t)t.nty * t.nzc * ns;
  t.per_xcd = (int)((t.nblocks + 7) / 8);
  const dim3 grid((unsigned)(t.per_xcd * 8));
  switch (t.kh) {
    case 2: hipLaunchKernelGGL((zhx_kernel<R, 2>), grid, dim3(t.threads), t.lds_bytes, s, a, t); break;
    case 3: hipLaunchKernelGGL((zhx_kernel<R, 3>), grid, dim3(t.threads), t.lds_bytes, s, a, t); break;
    case 4: hipLaunchKernelGGL((zhx_kernel<R, 4>), grid, dim3(t.threads), t.lds_bytes, s, a, t); break;
    default: return hipErrorInvalidConfiguration;
  }
  return hipGetLastError();
}

hipError_t launch_zhx(const ZHxArgs& a, int ns, hipStream_t s) {
  if (a.nd <= 0 || ns <= 0) return hipSuccess;
  if (a.r < 1 || a.r > kMaxRadius || a.n[0] > kZMaxThreads) return hipErrorInvalidValue;
  const ZTiling t = plan_zhx(a.n[0], a.n[1], a.n[2], ns, a.r);
  if (t.kh > 4 || t.lds_bytes > 96 * 1024) return hipErrorInvalidConfiguration;
  switch (a.r) {
    case 1: return launch_zhx_r<1>(a, t, ns, s);
    case 2: return launch_zhx_r<2>(a, t, ns, s);
    case 3: return launch_zhx_r<3>(a, t, ns, s);
    case 4: return launch_zhx_r<4>(a, t, ns, s);
    case 5: return launch_zhx_r<5>(a, t, ns, s);
    case 6: return launch_zhx_r<6>(a, t, ns, s);
    default: return hipErrorInvalidValue;
  }
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
