// hx_apply: matrix-free Kohn-Sham H on a block of orbitals, fused with the Chebyshev update.
//
// Sec. 2.1 applies H in three parts: the finite-difference Laplacian stencil of
// order n0 = 2r (3 n0 + 1 operations per output point), the pointwise Veff
// product and the Kleinman-Bylander projectors.  Here the stencil and Veff are one
// pass over HBM, and the Chebyshev three-term update of Alg. 1 (scaled form) is the
// epilogue, so one launch reads Y_k and Y_{k-1} once and writes Y_{k+1} once:
//
//   out[i] = sa * ((T + Veff) y - sc * y)[i] + sb * prev[i]
//
// Projector term: a point inside at most four projector entries (every point of the
// workloads with isolated atoms, ~90 % of the touched points with overlapping ones)
// is added in this pass from a 32/48-byte record holding its four alpha columns and
// chi values; each thread owns at most PY records per plane (a tile plane has at most
// PY * threads points), fetched one plane ahead with no dependent load and no inner
// loop.  The block's alpha row sits in LDS.  Points with more entries are left to
// nl_scatter, which adds theirs after this pass.
//
// Mapping on gfx950 (wave64, 160 KB LDS per CU, 8 XCDs with private L2):
//   * one block = one orbital x one tile of whole x-rows (nx wide, ty = nyg*PY
//     rows) x one chunk of z-planes; a thread owns PY consecutive y rows at one x;
//   * blocks are dealt to XCDs so that all tiles of one orbital and z chunk run on
//     the same XCD at about the same time: their halo rows hit the same L2;
//   * the block marches through z.  Each thread keeps its 2r+1 z-neighbours in a
//     register queue (the z part never touches LDS) and fetches the next plane one
//     iteration ahead.  The current plane of the tile plus r halo rows above and
//     below sits in LDS, double-buffered so one barrier per plane suffices; each LDS
//     row carries r halo columns on either side (periodic copies, or zeros for a
//     Dirichlet x), so every x neighbour is a fixed offset.  Besides its own elements
//     a thread stages KH values of the plane's halo rows and periodic x copies, each
//     read straight from its (wrapped) source; y neighbours are read once per column
//     and reused by the PY rows a thread owns.  The kernel is kept lean in registers:
//     on this path occupancy hides memory latency better than deeper per-thread
//     prefetch;
//   * global reads are buffer loads: a Dirichlet ghost is an out-of-range offset,
//     which returns zero without touching memory, so the loads need no branches.
#include "common.h"

#include <algorithm>

namespace chefsi {

constexpr unsigned kOOB = 0x80000000u;  // any buffer offset at or past the end reads as zero

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

__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void* p, int64_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, (int)bytes, 0x00020000);
}

// Buffer loads take a per-lane byte offset (voff) and a wave-uniform one (soff, a scalar
// register): the per-thread part of an address is computed once, the per-plane part on
// the scalar unit, so a load costs no vector instructions.  A lane whose voff is kOOB
// reads zero (kOOB + soff stays at or past the end because every buffer is below 2^31
// bytes and so is soff).
template <typename T>
__device__ __forceinline__ unsigned lane_off(int a) {
  return a < 0 ? kOOB : (unsigned)a * (unsigned)sizeof(T);
}

template <typename T>
__device__ __forceinline__ T bload(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff);
template <>
__device__ __forceinline__ double bload<double>(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
}
template <>
__device__ __forceinline__ float bload<float>(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0));
}

// The previous iterate and the output are each touched once per pass: in FP64 they are
// loaded and stored non-temporally (nt), which leaves more of the L2 to the halo rows and
// Veff that neighbouring blocks read again (72^3 FP64: 29.8 -> 29.0 ms of stencil passes
// per step; FP32 measured no gain and keeps the default policy).
template <typename T>
constexpr int kStreamPolicy = sizeof(T) == 8 ? 2 : 0;  // buffer cache policy bits: 2 = nt

template <typename T>
__device__ __forceinline__ T bload_stream(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff);
template <>
__device__ __forceinline__ double bload_stream<double>(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, kStreamPolicy<double>));
}
template <>
__device__ __forceinline__ float bload_stream<float>(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, kStreamPolicy<float>));
}
template <typename T>
__device__ __forceinline__ void bstore_stream(__amdgpu_buffer_rsrc_t r, T v, unsigned voff, unsigned soff);
template <>
__device__ __forceinline__ void bstore_stream<double>(__amdgpu_buffer_rsrc_t r, double v, unsigned voff,
                                                      unsigned soff) {
  typedef unsigned u32x2s __attribute__((ext_vector_type(2)));
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2s, v), r, voff, soff, kStreamPolicy<double>);
}
template <>
__device__ __forceinline__ void bstore_stream<float>(__amdgpu_buffer_rsrc_t r, float v, unsigned voff, unsigned soff) {
  __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, voff, soff, kStreamPolicy<float>);
}

template <typename T>
__device__ __forceinline__ void bstore(__amdgpu_buffer_rsrc_t r, T v, unsigned voff, unsigned soff);
template <>
__device__ __forceinline__ void bstore<double>(__amdgpu_buffer_rsrc_t r, double v, unsigned voff, unsigned soff) {
  typedef unsigned u32x2 __attribute__((__vector_size__(8)));
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, voff, soff, 0);
}
template <>
__device__ __forceinline__ void bstore<float>(__amdgpu_buffer_rsrc_t r, float v, unsigned voff, unsigned soff) {
  __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, voff, soff, 0);
}

// element at lane offset voff of plane po (element offset, uniform) of the nbytes-long
// array at p; po = -1 (a zero plane) selects a resource with no records: reads give zero
template <typename T>
__device__ __forceinline__ T pload(const T* p, int nbytes, unsigned voff, int po) {
  const __amdgpu_buffer_rsrc_t r = make_rsrc(p, po < 0 ? 0 : nbytes);
  return bload<T>(r, voff, po < 0 ? 0u : (unsigned)po * (unsigned)sizeof(T));
}

// one projector record (zeros when voff is kOOB): 32 bytes for FP32 values, 48 for FP64
template <typename TC>
__device__ __forceinline__ void load_rec(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff, int (&hdr)[3],
                                         TC (&v)[4]) {
  const auto h = __builtin_amdgcn_raw_buffer_load_b128(r, voff, soff, 0);
  const unsigned h0 = h[0], h1 = h[1], h2 = h[2];
  hdr[0] = (int)h0;
  hdr[1] = (int)h1;
  hdr[2] = (int)h2;
  const unsigned o1 = voff + 16u;
  if constexpr (sizeof(TC) == 4) {
    const auto w = __builtin_amdgcn_raw_buffer_load_b128(r, o1, soff, 0);
    const unsigned w0 = w[0], w1 = w[1], w2 = w[2], w3 = w[3];
    v[0] = __builtin_bit_cast(float, w0);
    v[1] = __builtin_bit_cast(float, w1);
    v[2] = __builtin_bit_cast(float, w2);
    v[3] = __builtin_bit_cast(float, w3);
  } else {
    const unsigned o2 = voff + 32u;
    const auto w = __builtin_amdgcn_raw_buffer_load_b128(r, o1, soff, 0);
    const auto u = __builtin_amdgcn_raw_buffer_load_b128(r, o2, soff, 0);
    v[0] = __builtin_bit_cast(double, (unsigned long long)w[0] | ((unsigned long long)w[1] << 32));
    v[1] = __builtin_bit_cast(double, (unsigned long long)w[2] | ((unsigned long long)w[3] << 32));
    v[2] = __builtin_bit_cast(double, (unsigned long long)u[0] | ((unsigned long long)u[1] << 32));
    v[3] = __builtin_bit_cast(double, (unsigned long long)u[2] | ((unsigned long long)u[3] << 32));
  }
}

// Number of LDS slots a block stages per plane besides its own body elements: the r halo
// rows above and below the tile (nx + 2r columns when x is periodic, the nx interior
// columns when it is not) and, when x is periodic, the r wrapped copies on each side of
// every body row.  (Dirichlet x halo columns are zeros written once.)
__host__ __device__ inline int hx_halo_slots(int nx, int ty, int radius, int per_x) {
  return 2 * radius * (per_x ? nx + 2 * radius : nx) + (per_x ? ty * 2 * radius : 0);
}

// Slot e of a plane's staged set: LDS destination (row-major with the given pitch, element
// x of a row at column r + x) and source row offset inside the plane (x added; -1 for a
// zero value).
__device__ __forceinline__ void halo_slot(int e, int nx, int ny, int ty, int y0, int radius, int pitch, int per_x,
                                          int per_y, int& dst, int& src) {
  const int w = per_x ? nx + 2 * radius : nx;
  int yy, c;
  if (e < 2 * radius * w) {  // halo rows: local rows [0, r) and [r + ty, ty + 2r)
    const int hr = e / w;
    c = e % w + (per_x ? 0 : radius);
    yy = hr < radius ? hr : hr + ty;
  } else {  // periodic x copies of the body rows: columns [0, r) and [r + nx, nx + 2r)
    const int f = e - 2 * radius * w;
    const int cc = f % (2 * radius);
    c = cc < radius ? cc : nx + cc;
    yy = radius + f / (2 * radius);
  }
  int gx = c - radius;
  if (gx < 0) gx += nx;  // only reached with periodic x (nx >= r: one wrap)
  if (gx >= nx) gx -= nx;
  dst = yy * pitch + c;
  src = row_offset(gx, y0 - radius + yy, nx, ny, per_y);
}

// one row per thread fits 128 VGPRs, so its blocks may hold 1024 threads (taller tiles,
// fewer halo rows per output row); two to four rows per thread keep 256 VGPRs and 512.
//
// The plane loop is kept free of divergent branches and of per-plane index arithmetic:
// every lane writes its LDS slots unconditionally (a lane with nothing to stage writes a
// dummy slot of its own past the end of the buffer), zero planes (Dirichlet z) are read
// through a resource with no records selected on the scalar unit, and the plane indices
// advance by one with a compare-and-reset wrap.
template <typename TI, typename TC, typename TO, int R, int PY, int KH, bool NL>
__global__ __launch_bounds__(hx_max_threads(PY)) void hx_apply_kernel(HxArgs<TI, TC, TO> a) {
  extern __shared__ __align__(16) unsigned char lds_raw[];
  constexpr int Q = 2 * R + 1;
  const int nx = a.nx, ny = a.ny, nz = a.nz;
  const int tid = threadIdx.x;
  const int nthr = blockDim.x;
  const int lane = tid & 63;

  // hardware deals consecutive block ids to the 8 XCDs in turn
  const int64_t logical = (int64_t)(blockIdx.x % 8) * a.per_xcd + blockIdx.x / 8;
  if (logical >= a.nblocks) return;
  const int per_vec = a.nty * a.nzc;
  const int64_t vec = logical / per_vec;
  const int rem = (int)(logical % per_vec);
  const int tile = rem % a.nty;
  const int zchunk = rem / a.nty;
  const int y0 = tile * a.ty;
  const int z0 = zchunk * a.zc;
  const int z1 = min(z0 + a.zc, nz);
  if (z0 >= nz) return;
  const int nzl = z1 - z0;

  const int plane_pts = a.ty * nx;
  // LDS tile rows carry r halo columns on each side (periodic copies, or zeros for a
  // Dirichlet x), so every x neighbour is a fixed offset from the thread's own element;
  // each buffer ends with 64 dummy slots (one per lane) for writes that have no target
  const int pitch = a.pitch;
  const int tile_elems = (a.ty + 2 * R) * pitch;
  const int tile_buf = tile_elems + kHxDummy;
  const int nl_buf = plane_pts + kHxDummy;
  // LDS: [record offsets of this chunk][alpha row][projector term x2] (NL only) [tile plane x2]
  int* s_rp = reinterpret_cast<int*>(lds_raw);
  const int rp_slots = NL ? ((nzl + 1 + 3) & ~3) : 0;
  TC* s_alpha = reinterpret_cast<TC*>(s_rp + rp_slots);
  const int al_slots = NL ? ((a.np_tot + 1) & ~1) : 0;
  TC* s_nl = s_alpha + al_slots;
  TI* s_tile = reinterpret_cast<TI*>(s_nl + (NL ? 2 * nl_buf : 0));
  typedef __attribute__((address_space(3))) const TC lds_tc;  // keeps the alpha reads ds_read
  lds_tc* l_alpha = (lds_tc*)s_alpha;

  const bool active = tid < nx * a.nyg;
  const int x = active ? tid % nx : 0;
  const int ly0 = active ? (tid / nx) * PY : 0;
  const int nplane = nx * ny;
  const TI* xv = a.x + vec * a.nd;
  const int xbytes = (int)(a.nd * (int64_t)sizeof(TI));
  const __amdgpu_buffer_rsrc_t rx = make_rsrc(xv, xbytes);
  const __amdgpu_buffer_rsrc_t rz = make_rsrc(xv, 0);  // no records: every load reads zero
  const unsigned xplane_bytes = (unsigned)nplane * (unsigned)sizeof(TI);
  const __amdgpu_buffer_rsrc_t rv = make_rsrc(a.veff, a.nd * (int64_t)sizeof(TC));
  // with no previous iterate the resource has no records: its loads read zero
  const bool has_prev = a.prev != nullptr;
  const __amdgpu_buffer_rsrc_t rp = make_rsrc(has_prev ? (const void*)(a.prev + vec * a.nd) : (const void*)a.out,
                                              has_prev ? a.nd * (int64_t)sizeof(TO) : 0);
  const __amdgpu_buffer_rsrc_t ro = make_rsrc(a.out + vec * a.nd, a.nd * (int64_t)sizeof(TO));
  const __amdgpu_buffer_rsrc_t rrec =
      make_rsrc(NL ? (const void*)a.rec : (const void*)a.out,
                NL ? (int64_t)a.rec_ptr[a.nty * nz] * (int64_t)sizeof(HxRec<TC>) : 0);
  // records of the plane being finished (hc, vc) and of the next one (hn, vn), PY per thread
  int hc[PY][3], hn[PY][3];
  TC vc[PY][4], vn[PY][4];
  if (NL) {
    const TC* g_alpha = a.alpha + vec * a.np_tot;
    for (int i = tid; i <= nzl; i += nthr) s_rp[i] = a.rec_ptr[tile * nz + z0 + i];
    for (int i = tid; i < a.np_tot; i += nthr) s_alpha[i] = g_alpha[i];
    for (int i = tid; i < 2 * nl_buf; i += nthr) s_nl[i] = TC(0);
    __syncthreads();
    const int rb = __builtin_amdgcn_readfirstlane(s_rp[0]), re = __builtin_amdgcn_readfirstlane(s_rp[1]);
#pragma unroll
    for (int r = 0; r < PY; ++r) {
      const int i = tid + r * nthr;
      load_rec<TC>(rrec, rb + i < re ? (unsigned)i * (unsigned)sizeof(HxRec<TC>) : kOOB,
                   (unsigned)rb * (unsigned)sizeof(HxRec<TC>), hc[r], vc[r]);
    }
  }

  // the thread's rows: plane offset (kOOB lane offsets for zero rows and rows past ny) and
  // LDS slot (a dummy slot for idle lanes)
  unsigned vq[PY], vv[PY], vp[PY];
  int sown[PY];
#pragma unroll
  for (int j = 0; j < PY; ++j) {
    const int gy = y0 + ly0 + j;
    const int ro_ = active ? row_offset(x, gy, nx, ny, a.per_y) : -1;
    const bool valid = active && gy < ny;
    vq[j] = lane_off<TI>(ro_);
    vv[j] = lane_off<TC>(valid ? ro_ : -1);
    vp[j] = lane_off<TO>(valid ? ro_ : -1);
    sown[j] = active ? (R + ly0 + j) * pitch + R + x : tile_elems + lane;
  }
  // staged slots (halo rows and periodic x copies): LDS slot and source lane offset
  int sdst[KH];
  unsigned vh[KH];
  {
    const int nslots = hx_halo_slots(nx, a.ty, R, a.per_x);
#pragma unroll
    for (int k = 0; k < KH; ++k) {
      const int e = tid + k * nthr;
      int dst = tile_elems + lane, src = -1;
      if (e < nslots) halo_slot(e, nx, ny, a.ty, y0, R, pitch, a.per_x, a.per_y, dst, src);
      sdst[k] = dst;
      vh[k] = lane_off<TI>(src);
    }
  }

  // q[s][j] = plane (z - R + s); pf = plane z + R (fetched one plane ahead); hp = staged
  // values of plane z
  TI q[Q][PY], pf[PY], hp[KH];
#pragma unroll
  for (int j = 0; j < PY; ++j) q[0][j] = TI(0);
#pragma unroll
  for (int s = 1; s < Q; ++s) {
    const int po = plane_offset(z0 - R - 1 + s, nplane, nz, a.per_z);
#pragma unroll
    for (int j = 0; j < PY; ++j) q[s][j] = pload<TI>(xv, xbytes, vq[j], po);
  }
  {
    const int po = plane_offset(z0 + R, nplane, nz, a.per_z);
#pragma unroll
    for (int j = 0; j < PY; ++j) pf[j] = pload<TI>(xv, xbytes, vq[j], po);
    const int ph = plane_offset(z0, nplane, nz, a.per_z);
#pragma unroll
    for (int k = 0; k < KH; ++k) hp[k] = pload<TI>(xv, xbytes, vh[k], ph);
  }

  if (!a.per_x) {  // Dirichlet x: the halo columns of both tile buffers (never staged) hold zeros
    const int nrows = 2 * (a.ty + 2 * R);
    for (int i = tid; i < nrows * 2 * R; i += nthr) {
      const int row = i / (2 * R), c = i % (2 * R);
      const int buf = row / (a.ty + 2 * R), rr = row % (a.ty + 2 * R);
      s_tile[buf * tile_buf + rr * pitch + (c < R ? c : nx + c)] = TI(0);
    }
  }

  // planes fetched inside the loop: the queue's z + R + 1 and the staged set's z + 1,
  // advanced by one per plane (wrapped when z is periodic; a Dirichlet plane at or past
  // nz reads zero)
  int pb = z0 + R + 1, ph = z0 + 1;
  if (a.per_z) {
    pb %= nz;
    ph %= nz;
  }
  for (int zl = 0; zl < nzl; ++zl) {
    const int z = z0 + zl;
    TI* tl = s_tile + (zl & 1) * tile_buf;
    const bool more = zl + 1 < nzl;
    if (NL) {  // records of plane zl + 1
      const int rb = more ? __builtin_amdgcn_readfirstlane(s_rp[zl + 1]) : 0;
      const int re = more ? __builtin_amdgcn_readfirstlane(s_rp[zl + 2]) : 0;
#pragma unroll
      for (int r = 0; r < PY; ++r) {
        const int i = tid + r * nthr;
        load_rec<TC>(rrec, rb + i < re ? (unsigned)i * (unsigned)sizeof(HxRec<TC>) : kOOB,
                     (unsigned)rb * (unsigned)sizeof(HxRec<TC>), hn[r], vn[r]);
      }
    }
    // Veff and previous iterate of this plane, used at the end of the iteration
    TC cv[PY], cp[PY];
    const unsigned zo = (unsigned)(nplane * z);
#pragma unroll
    for (int j = 0; j < PY; ++j) {
      cv[j] = bload<TC>(rv, vv[j], zo * (unsigned)sizeof(TC));
      cp[j] = TC(bload_stream<TO>(rp, vp[j], zo * (unsigned)sizeof(TO)));
    }
    // advance the queue; fetch plane z + R + 1
#pragma unroll
    for (int s = 0; s < Q - 1; ++s)
#pragma unroll
      for (int j = 0; j < PY; ++j) q[s][j] = q[s + 1][j];
#pragma unroll
    for (int j = 0; j < PY; ++j) q[Q - 1][j] = pf[j];
    {
      const bool ok = more && pb < nz;
      const __amdgpu_buffer_rsrc_t r = ok ? rx : rz;
      const unsigned so = ok ? (unsigned)pb * xplane_bytes : 0u;
#pragma unroll
      for (int j = 0; j < PY; ++j) pf[j] = bload<TI>(r, vq[j], so);
    }
    // stage plane z in LDS; fetch the staged set of plane z + 1
#pragma unroll
    for (int j = 0; j < PY; ++j) tl[sown[j]] = q[R][j];
#pragma unroll
    for (int k = 0; k < KH; ++k) tl[sdst[k]] = hp[k];
    {
      const bool ok = more && ph < nz;
      const __amdgpu_buffer_rsrc_t r = ok ? rx : rz;
      const unsigned so = ok ? (unsigned)ph * xplane_bytes : 0u;
#pragma unroll
      for (int k = 0; k < KH; ++k) hp[k] = bload<TI>(r, vh[k], so);
    }
    ++pb;
    ++ph;
    if (a.per_z) {
      pb = pb == nz ? 0 : pb;
      ph = ph == nz ? 0 : ph;
    }
    TC* nla = s_nl + (zl & 1) * nl_buf;
    if (NL) {  // projector term of plane zl into its (zeroed) accumulator, one writer per point
      const int nrec = s_rp[zl + 1] - s_rp[zl];
#pragma unroll
      for (int r = 0; r < PY; ++r) {
        const int dst = tid + r * nthr < nrec ? hc[r][0] : plane_pts + lane;
        const unsigned c01 = (unsigned)hc[r][1], c23 = (unsigned)hc[r][2];
        nla[dst] = vc[r][0] * l_alpha[c01 & 0xffffu] + vc[r][1] * l_alpha[c01 >> 16] +
                   vc[r][2] * l_alpha[c23 & 0xffffu] + vc[r][3] * l_alpha[c23 >> 16];
      }
    }
    __syncthreads();

    TC acc[PY];
#pragma unroll
    for (int j = 0; j < PY; ++j) {
      TC t = a.c0 * TC(q[R][j]);
#pragma unroll
      for (int p = 1; p <= R; ++p) t += a.cz[p] * (TC(q[R + p][j]) + TC(q[R - p][j]));
      acc[j] = t;
    }
    // y part: each LDS row of the column is read once and feeds every row it neighbours
#pragma unroll
    for (int t = 0; t < PY + 2 * R; ++t) {
      const TC v = TC(tl[(ly0 + t) * pitch + R + x]);
#pragma unroll
      for (int j = 0; j < PY; ++j) {
        const int p = t - R - j;
        if (p != 0 && p >= -R && p <= R) acc[j] += a.cy[p < 0 ? -p : p] * v;
      }
    }
    // x part: neighbours inside the row
#pragma unroll
    for (int j = 0; j < PY; ++j) {
      const TI* row = tl + (R + ly0 + j) * pitch + R + x;
      TC t = TC(0);
#pragma unroll
      for (int p = 1; p <= R; ++p) t += a.cx[p] * (TC(row[p]) + TC(row[-p]));
      acc[j] += t;
    }
#pragma unroll
    for (int j = 0; j < PY; ++j) {
      const TC v = TC(q[R][j]);
      TC hy = acc[j] + cv[j] * v;
      if (NL) {
        const int li = active ? (ly0 + j) * nx + x : plane_pts + lane;
        hy += nla[li];
        nla[li] = TC(0);
      }
      // idle lanes and rows past ny store through a kOOB offset: no write
      bstore_stream<TO>(ro, TO(a.sa * (hy - a.sc * v) + a.sb * cp[j]), vp[j], zo * (unsigned)sizeof(TO));
    }
    if (NL) {
#pragma unroll
      for (int r = 0; r < PY; ++r) {
#pragma unroll
        for (int k = 0; k < 3; ++k) hc[r][k] = hn[r][k];
#pragma unroll
        for (int k = 0; k < 4; ++k) vc[r][k] = vn[r][k];
      }
    }
  }
}

size_t hx_lds_bytes(const HxPlan& p, int nx, int radius, int elem_bytes, int np_tot, int acc_bytes) {
  size_t lds = 2 * ((size_t)(p.ty + 2 * radius) * hx_pitch(nx, radius, elem_bytes, p.py) + kHxDummy) * elem_bytes;
  if (np_tot >= 0) {
    lds += (size_t)((p.zc + 1 + 3) & ~3) * sizeof(int);
    lds += (size_t)((np_tot + 1) & ~1) * acc_bytes;
    lds += 2 * ((size_t)p.ty * nx + kHxDummy) * acc_bytes;
  }
  return lds;
}

HxPlan plan_hx(int nx, int ny, int nz, int ns, int radius, int elem_bytes, int py_override, int nyg_override) {
  // Cost of a tiling, fitted to measured launches on 72^3 and 120^3 grids (FP64 and FP32):
  // idle lanes and rows beyond ny waste work, halo rows cost reads, blocks above 512
  // threads and two rows per thread cost occupancy (more so in FP32 for the former and in
  // FP64 for the latter).  Tiles of at least r+1 rows are required when any fit (thinner
  // ones read the halo more than twice per output row and measured far slower).
  HxPlan best;
  double best_cost = 1e300;
  bool best_tall = false;
  const double big_block = elem_bytes == 8 ? 1.2 : 1.35;
  const double two_rows = elem_bytes == 8 ? 1.3 : 1.2;
  // Three or four rows per thread are reached by an explicit tiling or the timed autotune
  // only: the cost model was fitted to one and two (in FP32 three rows measured 2-7% faster
  // on the 72^3 and 60x60x180 mixed filters, four at 120^3; in FP64 their register queue
  // costs occupancy).
  const int pys[] = {1, 2, 3, 4};
  for (int py : pys) {
    if (py_override > 0 ? py != py_override : py > 2) continue;
    for (int nyg = 1; nx * nyg <= hx_max_threads(py); ++nyg) {
      if (nyg_override > 0 && nyg != nyg_override) continue;
      const int ty = nyg * py;
      const int nty = (ny + ty - 1) / ty;
      const int threads = nx * nyg;
      const int waves = (threads + 63) / 64;
      // staged values per thread bound (counted for a periodic x, the larger set)
      const int nslots = hx_halo_slots(nx, ty, radius, 1);
      if (nslots > kHxMaxHalo * waves * 64) continue;
      const size_t lds = 2 * ((size_t)(ty + 2 * radius) * hx_pitch(nx, radius, elem_bytes, py) + kHxDummy) * elem_bytes;
      if (lds > 48 * 1024) continue;
      const double lane_eff = (double)threads / (waves * 64.0);
      const double row_eff = (double)ny / (nty * ty);
      const double halo = (double)(ty + 2 * radius) / ty;
      double cost = 1.0 / (lane_eff * row_eff) * (1.0 + 0.15 * (halo - 1.0));
      if (threads > 512) cost *= big_block;
      if (py >= 2) cost *= two_rows;
      if (threads < 128) cost *= 1.15;
      if (ty > ny + 2 * radius) cost *= 2.0;
      const bool tall = ty >= std::min(radius + 1, ny);
      if ((tall && !best_tall) || (tall == best_tall && cost < best_cost - 1e-12)) {
        best_tall = tall;
        best_cost = cost;
        best.ok = true;
        best.py = py;
        best.nyg = nyg;
        best.ty = ty;
        best.nty = nty;
        best.threads = waves * 64;
        best.kh = std::max(2, (nslots + waves * 64 - 1) / (waves * 64));
        best.lds_tile_bytes = lds;
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

template <typename TI, typename TC, typename TO, int R, int PY, int KH, bool NL>
static hipError_t launch_final(const HxArgs<TI, TC, TO>& a0, const HxPlan& p, int ns, hipStream_t s) {
  HxArgs<TI, TC, TO> a = a0;
  a.nyg = p.nyg;
  a.ty = p.ty;
  a.nty = p.nty;
  a.zc = p.zc;
  a.nzc = p.nzc;
  a.nblocks = (int64_t)p.nty * p.nzc * ns;
  a.pitch = hx_pitch(a.nx, R, (int)sizeof(TI), PY);
  a.per_xcd = (int)((a.nblocks + 7) / 8);
  const size_t lds = hx_lds_bytes(p, a.nx, R, (int)sizeof(TI), NL ? a.np_tot : -1, (int)sizeof(TC));
  if (lds > kHxMaxLds) return hipErrorInvalidConfiguration;
  dim3 grid((unsigned)(a.per_xcd * 8));
  hipLaunchKernelGGL((hx_apply_kernel<TI, TC, TO, R, PY, KH, NL>), grid, dim3(p.threads), lds, s, a);
  return hipGetLastError();
}

template <typename TI, typename TC, typename TO, int R, int PY>
static hipError_t launch_rp(const HxArgs<TI, TC, TO>& a, const HxPlan& p, int ns, hipStream_t s) {
  const bool nl = a.rec_ptr != nullptr;
  switch (p.kh) {
    case 2:
      return nl ? launch_final<TI, TC, TO, R, PY, 2, true>(a, p, ns, s) : launch_final<TI, TC, TO, R, PY, 2, false>(a, p, ns, s);
    case 3:
      return nl ? launch_final<TI, TC, TO, R, PY, 3, true>(a, p, ns, s) : launch_final<TI, TC, TO, R, PY, 3, false>(a, p, ns, s);
    case 4:
      return nl ? launch_final<TI, TC, TO, R, PY, 4, true>(a, p, ns, s) : launch_final<TI, TC, TO, R, PY, 4, false>(a, p, ns, s);
    default:
      return hipErrorInvalidValue;
  }
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
