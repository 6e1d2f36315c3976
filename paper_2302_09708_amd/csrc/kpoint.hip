// H at a Bloch wavevector k on complex FP64 orbitals (interleaved re/im, Nd x Ns column
// major): Sec. 2 of the paper runs every Brillouin-zone sample other than Gamma in complex
// double precision.  Kernels, launched in this order on one stream:
//   zhx       out = sa ((T_k + Veff) x - sc x) + sb prev    (Bloch-phased FD ghosts)
//   zband     out[v, p] += sa sum_{e in entries of p} chi~[e] alpha[col[e], v] at every
//             touched point p, then the slot partials of the next coefficients,
//             sum over the region's points of q of conj(chi~) out[v, p]
//   zband_reduce  alpha[q, v] = gamma_q dV * (sum of q's slot partials, region order)
// (a gather-only zband pass forms the coefficients of a block that no pass has produced).
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

// ---------------------------------------------------------------------------
// zband: the complex counterpart of the real band pass.  One block per (region, run of
// orbital groups of kZG orbitals), one thread per point; the region's entry tables sit in
// LDS for the whole run; the next group's point values and staged coefficients are fetched
// into registers while the current group is scattered and gathered.
// ---------------------------------------------------------------------------
constexpr int kZG = 4;  // orbitals per group: 512 points x 4 x 16 B = 32 KB of LDS

template <bool SCATTER>
__global__ __launch_bounds__(kBandThreads) void zband_kernel(ZNbArgs a, int gather) {
  constexpr int AJ = (kBandMaxSlots * kZG + kBandThreads - 1) / kBandThreads;
  __shared__ double2 ys[kBandMaxPts * kZG];
  __shared__ double2 as[kBandMaxSlots * kZG];
  __shared__ double2 echi[kZBandMaxEnt];
  __shared__ double2 gchi[kZBandMaxEnt];
  __shared__ unsigned short els[kZBandMaxEnt];
  __shared__ unsigned short gloc[kZBandMaxEnt];
  __shared__ int sent[kBandMaxSlots + 1];
  __shared__ int sq[kBandMaxSlots];
  const int64_t logical = (int64_t)(blockIdx.x % 8) * a.per_xcd + blockIdx.x / 8;
  if (logical >= (int64_t)a.nreg * a.nchunks) return;
  const int reg = (int)(logical / a.nchunks);
  const int g0 = (int)(logical % a.nchunks) * a.gpc;
  const int g1 = min(a.ngroups, g0 + a.gpc);
  if (g0 >= g1) return;
  const int tid = threadIdx.x;
  const int p0 = a.reg_pt[reg], np = a.reg_pt[reg + 1] - p0;
  const int s0 = a.reg_slot[reg], nslot = a.reg_slot[reg + 1] - s0;
  const int eb = a.pt_ent[p0];
  if (SCATTER) {
    const int ne = a.pt_ent[p0 + np] - eb;
    for (int e = tid; e < ne; e += kBandThreads) {
      echi[e] = a.ent_chi[eb + e];
      els[e] = (unsigned short)a.ent_ls[eb + e];
    }
  }
  const int gb = a.slot_ent[s0];
  if (gather) {
    const int ne = a.slot_ent[s0 + nslot] - gb;
    for (int e = tid; e < ne; e += kBandThreads) {
      gchi[e] = a.gent_chi[gb + e];
      gloc[e] = (unsigned short)a.gent_loc[gb + e];
    }
  }
  for (int sl = tid; sl <= nslot; sl += kBandThreads) sent[sl] = a.slot_ent[s0 + sl] - gb;
  for (int sl = tid; sl < nslot; sl += kBandThreads) sq[sl] = a.slot_q[s0 + sl];
  const bool own = tid < np;
  int64_t pi = 0;
  int e0 = 0, e1 = 0;
  if (own) {
    pi = a.pt_idx[p0 + tid];
    e0 = a.pt_ent[p0 + tid] - eb;
    e1 = a.pt_ent[p0 + tid + 1] - eb;
  }
  const int nitem = nslot * kZG;
  // register values as separate real and imaginary arrays (kept in registers)
  auto load_y = [&](int g, double (&yr)[kZG], double (&yi)[kZG]) {
    const int v0 = g * kZG;
#pragma unroll
    for (int u = 0; u < kZG; ++u) {
      double2 v = make_double2(0.0, 0.0);
      if (own && v0 + u < a.ns) v = a.y[(int64_t)(v0 + u) * a.nd + pi];
      yr[u] = v.x;
      yi[u] = v.y;
    }
  };
  auto load_alpha = [&](int g, double (&ar)[AJ], double (&ai)[AJ]) {
    const int v0 = g * kZG;
#pragma unroll
    for (int j = 0; j < AJ; ++j) {
      const int it = tid + j * kBandThreads, ls = it / kZG, u = it % kZG;
      double2 v = make_double2(0.0, 0.0);
      if (it < nitem && v0 + u < a.ns) v = a.alpha[(int64_t)sq[ls] * a.ns + v0 + u];
      ar[j] = v.x;
      ai[j] = v.y;
    }
  };
  auto stage_alpha = [&](const double (&ar)[AJ], const double (&ai)[AJ]) {
#pragma unroll
    for (int j = 0; j < AJ; ++j) {
      const int it = tid + j * kBandThreads;
      if (it < nitem) as[it] = make_double2(ar[j], ai[j]);
    }
  };
  __syncthreads();  // slot columns staged
  double ycr[kZG], yci[kZG], ynr[kZG], yni[kZG], anr[AJ], ani[AJ];
  load_y(g0, ycr, yci);
  if (SCATTER) {
    load_alpha(g0, anr, ani);
    stage_alpha(anr, ani);
  }
  __syncthreads();
  for (int g = g0; g < g1; ++g) {
    const int v0 = g * kZG, nv = min(kZG, a.ns - v0);
    const bool more = g + 1 < g1;
    if (more) {
      load_y(g + 1, ynr, yni);
      if (SCATTER) load_alpha(g + 1, anr, ani);
    }
    if (own) {
      if (SCATTER) {
        double tr[kZG], ti[kZG];
#pragma unroll
        for (int u = 0; u < kZG; ++u) tr[u] = ti[u] = 0.0;
        for (int e = e0; e < e1; ++e) {
          const double2 c = echi[e];
          const double2* al = as + els[e] * kZG;
#pragma unroll
          for (int u = 0; u < kZG; ++u) {
            const double2 m = cmul(c, al[u]);
            tr[u] += m.x;
            ti[u] += m.y;
          }
        }
#pragma unroll
        for (int u = 0; u < kZG; ++u) {
          ycr[u] += a.sa * tr[u];
          yci[u] += a.sa * ti[u];
          if (u < nv) a.y[(int64_t)(v0 + u) * a.nd + pi] = make_double2(ycr[u], yci[u]);
        }
      }
#pragma unroll
      for (int u = 0; u < kZG; ++u) ys[tid * kZG + u] = make_double2(ycr[u], yci[u]);
    }
    __syncthreads();  // ys complete; the staged coefficients are no longer read
    if (SCATTER && more) stage_alpha(anr, ani);
    if (gather) {
      // slot partials: one thread per (slot, orbital), the slot's entries in index order
      for (int it = tid; it < nitem; it += kBandThreads) {
        const int sl = it / kZG, u = it % kZG;
        if (u >= nv) continue;
        // four running sums over entries e = 4 m + c (independent LDS chains), added in a
        // fixed order
        double sr[4] = {0.0, 0.0, 0.0, 0.0}, si[4] = {0.0, 0.0, 0.0, 0.0};
        const int eb0 = sent[sl], ee = sent[sl + 1];
        int e = eb0;
        for (; e + 4 <= ee; e += 4) {
#pragma unroll
          for (int c = 0; c < 4; ++c) {
            const double2 m = cmul(gchi[e + c], ys[gloc[e + c] * kZG + u]);
            sr[c] += m.x;
            si[c] += m.y;
          }
        }
        for (int c = 0; e < ee; ++e, ++c) {
          const double2 m = cmul(gchi[e], ys[gloc[e] * kZG + u]);
          sr[c] += m.x;
          si[c] += m.y;
        }
        a.partial[(int64_t)(s0 + sl) * a.ns + v0 + u] =
            make_double2((sr[0] + sr[1]) + (sr[2] + sr[3]), (si[0] + si[1]) + (si[2] + si[3]));
      }
    }
    __syncthreads();  // ys free, next coefficients staged
#pragma unroll
    for (int u = 0; u < kZG; ++u) {
      ycr[u] = ynr[u];
      yci[u] = yni[u];
    }
  }
}

// alpha[q][v] = gdv[q] * sum over the slots of q (region order) of partial[slot][v]
__global__ __launch_bounds__(256) void zband_reduce_kernel(const double2* __restrict__ partial,
                                                           const int* __restrict__ q_slot_ptr,
                                                           const int* __restrict__ q_slot,
                                                           const double* __restrict__ gdv, int np_tot, int ns,
                                                           double2* __restrict__ alpha) {
  const int q = blockIdx.y;
  const int v = blockIdx.x * 256 + threadIdx.x;
  if (q >= np_tot || v >= ns) return;
  double re = 0.0, im = 0.0;
  for (int k = q_slot_ptr[q]; k < q_slot_ptr[q + 1]; ++k) {
    const double2 t = partial[(int64_t)q_slot[k] * ns + v];
    re += t.x;
    im += t.y;
  }
  alpha[(int64_t)q * ns + v] = make_double2(gdv[q] * re, gdv[q] * im);
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

hipError_t launch_zband(const ZNbArgs& a0, bool scatter, bool gather, hipStream_t s) {
  if (a0.nreg <= 0 || a0.ns <= 0) return hipSuccess;
  ZNbArgs a = a0;
  a.ngroups = (a.ns + kZG - 1) / kZG;
  // runs of groups: about 4096 blocks in all, each run as long as that allows
  const int want = (int)std::min<int64_t>(a.ngroups, std::max<int64_t>(1, (4096 + a.nreg - 1) / a.nreg));
  a.gpc = (a.ngroups + want - 1) / want;
  a.nchunks = (a.ngroups + a.gpc - 1) / a.gpc;
  const int64_t nb = (int64_t)a.nreg * a.nchunks;
  a.per_xcd = (int)((nb + 7) / 8);
  const dim3 grid((unsigned)(a.per_xcd * 8));
  if (scatter)
    hipLaunchKernelGGL(zband_kernel<true>, grid, dim3(kBandThreads), 0, s, a, gather ? 1 : 0);
  else
    hipLaunchKernelGGL(zband_kernel<false>, grid, dim3(kBandThreads), 0, s, a, 1);
  return hipGetLastError();
}

hipError_t launch_zband_reduce(const double2* partial, const int* q_slot_ptr, const int* q_slot, const double* gdv,
                               int np_tot, int ns, double2* alpha, hipStream_t s) {
  if (np_tot <= 0 || ns <= 0) return hipSuccess;
  const dim3 grid((unsigned)((ns + 255) / 256), (unsigned)np_tot);
  hipLaunchKernelGGL(zband_reduce_kernel, grid, dim3(256), 0, s, partial, q_slot_ptr, q_slot, gdv, np_tot, ns, alpha);
  return hipGetLastError();
}

}  // namespace chefsi
