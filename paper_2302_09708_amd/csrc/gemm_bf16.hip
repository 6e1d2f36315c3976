// Split-bf16 contractions of the mixed-precision projection and rotation (gfx950 MFMA).
//
// Each FP32 operand value x is written as x = hi + lo + O(2^-17 |x|) with
// hi = bf16(x) and lo = bf16(x - hi) (round to nearest even), and a product as
// a b ~ a_hi b_hi + a_hi b_lo + a_lo b_hi: three bf16 MFMAs with FP32
// accumulation, error about 2^-15 |a b| per product (the dropped a_lo b_lo term
// and the two representation errors).  The Cholesky of Ms, the eigensolve and the
// final Rayleigh-Ritz pass stay in FP64 elsewhere.
//
// v_mfma_f32_32x32x16_bf16 lane layout (measured): A[i][k] comes from lane
// i + 32 (k / 8), element k % 8; B[k][j] from lane j + 32 (k / 8), element k % 8;
// D[i][j] lands in lane j + 32 ((i / 4) % 2), register 4 (i / 8) + i % 4, i.e.
// lane l, register v holds row 8 (v / 4) + 4 (l / 32) + v % 4, column l % 32.
//
// Projection (Alg. 1; Sec. 2.2): partial[split][tile] = A(:, I)^T B(:, J) over one
//   K chunk, 128 x 128 upper tiles, the same split-K plan and partial layout as the
//   FP64 kernel (so the FP64 fixed-order reduction is shared).  Both operands are
//   contiguous along K, so 32-wide K stages of both tiles are split into hi/lo and
//   staged through double-buffered LDS (one barrier per stage).
// Rotation (Alg. 1; Sec. 2.4): O = X Z computed as O^T = Z^T X^T.  Z is split once
//   into bf16 hi/lo arrays (zero padded, so the K tail needs no masking); a block
//   stages a 128-column slice of Z through LDS and every wave gathers the MFMA B
//   operand straight from X: lane l reads grid point p = l % 32 of 8 consecutive
//   columns, so each load instruction covers 128 contiguous bytes of two columns and
//   no transpose is needed.  Results leave as 128-byte rows of O.
#include "common.h"

#include <algorithm>

namespace chefsi {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef unsigned u32x4 __attribute__((ext_vector_type(4)));
typedef float f32x4u __attribute__((ext_vector_type(4), aligned(4)));  // rows of odd length are only 4-byte aligned

namespace {

constexpr int kT = 128;        // projection block tile (both dimensions)
constexpr int kKS = 32;        // K per stage
constexpr int kLd = kKS + 8;   // LDS row stride in bf16 (80 bytes: conflict-free 16-byte reads)
constexpr int kRotJ = 128;     // rotation: output columns per block
constexpr int kRotP = 256;     // rotation: grid points per block (64 per wave)
constexpr int kSubStages = 512;  // projection: K stages summed in FP32 before an FP64 flush (16384 rows)


__device__ __forceinline__ f32x16 mfma_bf16(bf16x8 a, bf16x8 b, f32x16 c) {
  return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
}

// x = hi + lo with hi = bf16(x), lo = bf16(x - hi), both round-to-nearest-even.
__device__ __forceinline__ void split_bf16(float x, __bf16& hi, __bf16& lo) {
  hi = (__bf16)x;
  lo = (__bf16)(x - (float)hi);
}

__device__ __forceinline__ void split8(const float (&x)[8], bf16x8& hi, bf16x8& lo) {
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    __bf16 h, l;
    split_bf16(x[e], h, l);
    hi[e] = h;
    lo[e] = l;
  }
}

__device__ __forceinline__ u32x4 as_u4(bf16x8 v) { return __builtin_bit_cast(u32x4, v); }
__device__ __forceinline__ bf16x8 as_bf8(u32x4 v) { return __builtin_bit_cast(bf16x8, v); }

__device__ __forceinline__ void upper_tile_of(int t, int nt, int& ti, int& tj) {
  int i = 0;
  int row = nt;
  while (t >= row) {
    t -= row;
    ++i;
    --row;
  }
  ti = i;
  tj = i + t;
}

}  // namespace

// ---------------------------------------------------------------------------
// Projection partial tiles.
// ---------------------------------------------------------------------------
struct GramStage {
  float a[16];
  float b[16];
};

// Thread t stages row t / 2 of both tiles: the 16 elements k .. k + 15 (k = stage start
// + 16 (t % 2)) of rows pa and pb; elements at or past ke read as zero unless full.
__device__ __forceinline__ void gram_load(GramStage& st, const float* __restrict__ pa, const float* __restrict__ pb,
                                          int64_t k, int64_t ke, bool full) {
  if (full) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const f32x4u va = *reinterpret_cast<const f32x4u*>(pa + k + 4 * q);
      const f32x4u vb = *reinterpret_cast<const f32x4u*>(pb + k + 4 * q);
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        st.a[4 * q + e] = va[e];
        st.b[4 * q + e] = vb[e];
      }
    }
  } else {
#pragma unroll
    for (int e = 0; e < 16; ++e) {
      const bool ok = k + e < ke;
      st.a[e] = ok ? pa[k + e] : 0.f;
      st.b[e] = ok ? pb[k + e] : 0.f;
    }
  }
}

__device__ __forceinline__ void gram_store_lds(const GramStage& st, __bf16* ah, __bf16* al, __bf16* bh, __bf16* bl,
                                               int off) {
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    float xa[8], xb[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      xa[e] = st.a[8 * q + e];
      xb[e] = st.b[8 * q + e];
    }
    bf16x8 h, l;
    split8(xa, h, l);
    *reinterpret_cast<u32x4*>(ah + off + 8 * q) = as_u4(h);
    *reinterpret_cast<u32x4*>(al + off + 8 * q) = as_u4(l);
    split8(xb, h, l);
    *reinterpret_cast<u32x4*>(bh + off + 8 * q) = as_u4(h);
    *reinterpret_cast<u32x4*>(bl + off + 8 * q) = as_u4(l);
  }
}

// FP32 accumulators of a wave's 64 x 64 part into the FP64 partial tile (added to what the
// same threads stored before when `add`), then cleared.  One writer per element, fixed order.
__device__ __forceinline__ void flush_tile(f32x16 (&acc)[2][2], double* __restrict__ pt, int wm, int wn, int g,
                                           int r32, bool add) {
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const int ii = wm * 64 + i * 32 + 8 * (v >> 2) + 4 * g + (v & 3);
        const int jj = wn * 64 + j * 32 + r32;
        double* q = pt + ii * kT + jj;
        *q = add ? *q + (double)acc[i][j][v] : (double)acc[i][j][v];
        acc[i][j][v] = 0.f;
      }
}

// two blocks per CU (80 KB of LDS each, at most 256 registers per lane): a second wave on
// every SIMD hides the global-load and LDS latency of the other (measured 14-22 % faster
// than one wave per SIMD on 72^3 to 120^3 blocks)
__global__ __launch_bounds__(256, 2) void gram_bf16x3_kernel(const float* __restrict__ A, const float* __restrict__ B,
                                                          int64_t nd, int ns, int nt, int ntiles, int64_t kchunk,
                                                          double* __restrict__ partial) {
  // [buffer][hi A, lo A, hi B, lo B][128 rows][kLd]
  __shared__ __attribute__((aligned(16))) __bf16 lds[2][4][kT * kLd];
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm = wave & 1, wn = wave >> 1;
  const int tile = blockIdx.x % ntiles;
  const int split = blockIdx.x / ntiles;
  int ti, tj;
  upper_tile_of(tile, nt, ti, tj);
  const int64_t kb = (int64_t)split * kchunk;
  const int64_t ke = min(nd, kb + kchunk);

  const int lrow = tid >> 1;       // staged row
  const int lhalf = tid & 1;       // staged K half
  const int ra = min(ti * kT + lrow, ns - 1);
  const int rb = min(tj * kT + lrow, ns - 1);
  const float* pa = A + (int64_t)ra * nd;
  const float* pb = B + (int64_t)rb * nd;
  const int st_off = lrow * kLd + 16 * lhalf;

  f32x16 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int v = 0; v < 16; ++v) acc[i][j][v] = 0.f;

  const int nstage = (int)((ke - kb + kKS - 1) / kKS);
  // partial tile, row-major 128 x 128: element (ii, jj) at ii * 128 + jj
  double* pt = partial + ((int64_t)split * ntiles + tile) * (kT * kT);
  GramStage st;
  if (nstage > 0) {
    gram_load(st, pa, pb, kb + 16 * lhalf, ke, kb + kKS <= ke);
    gram_store_lds(st, lds[0][0], lds[0][1], lds[0][2], lds[0][3], st_off);
  }
  __syncthreads();

  const int r32 = lane & 31, g = lane >> 5;
  for (int t = 0; t < nstage; ++t) {
    const int buf = t & 1;
    const bool more = t + 1 < nstage;
    const int64_t kn = kb + (int64_t)(t + 1) * kKS;
    if (more) gram_load(st, pa, pb, kn + 16 * lhalf, ke, kn + kKS <= ke);
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      bf16x8 ah[2], al[2], bh[2], bl[2];
#pragma unroll
      for (int f = 0; f < 2; ++f) {
        const int oa = (wm * 64 + f * 32 + r32) * kLd + 16 * s + 8 * g;
        const int ob = (wn * 64 + f * 32 + r32) * kLd + 16 * s + 8 * g;
        ah[f] = as_bf8(*reinterpret_cast<const u32x4*>(lds[buf][0] + oa));
        al[f] = as_bf8(*reinterpret_cast<const u32x4*>(lds[buf][1] + oa));
        bh[f] = as_bf8(*reinterpret_cast<const u32x4*>(lds[buf][2] + ob));
        bl[f] = as_bf8(*reinterpret_cast<const u32x4*>(lds[buf][3] + ob));
      }
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = mfma_bf16(al[i], bh[j], acc[i][j]);
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = mfma_bf16(ah[i], bl[j], acc[i][j]);
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = mfma_bf16(ah[i], bh[j], acc[i][j]);
    }
    if (more) gram_store_lds(st, lds[buf ^ 1][0], lds[buf ^ 1][1], lds[buf ^ 1][2], lds[buf ^ 1][3], st_off);
    // every kSubStages stages the FP32 sums move into the FP64 partial tile (FP32 sums span
    // at most kSubStages * kKS rows of K)
    if ((t + 1) % kSubStages == 0 && more) {
      flush_tile(acc, pt, wm, wn, g, r32, t + 1 > kSubStages);
    }
    __syncthreads();
  }
  flush_tile(acc, pt, wm, wn, g, r32, nstage > kSubStages);
}

hipError_t launch_gram_bf16x3(const float* A, const float* B, int64_t nd, int ns, const GramPlan& p,
                              double* partial, hipStream_t s) {
  if (p.tile != kT) return hipErrorInvalidValue;
  dim3 grid((unsigned)(p.ntiles * p.splits));
  hipLaunchKernelGGL(gram_bf16x3_kernel, grid, dim3(256), 0, s, A, B, nd, ns, p.nt, p.ntiles, p.kchunk, partial);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Rotation.
// ---------------------------------------------------------------------------
size_t zsplit_ld(int ns) { return (size_t)((ns + kKS - 1) / kKS) * kKS; }
size_t zsplit_cols(int ns) { return (size_t)((ns + kRotJ - 1) / kRotJ) * kRotJ; }
size_t zsplit_bytes(int ns) { return 2 * zsplit_cols(ns) * zsplit_ld(ns) * sizeof(__bf16); }

// zh/zl[j * ld + i] = split of Z[i + j ns] for i < ns, j < ns; zero in the padding.
__global__ void zsplit_kernel(const double* __restrict__ Z, int ns, int ld, int cols, __bf16* __restrict__ zh,
                              __bf16* __restrict__ zl) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)ld * cols) return;
  const int i = (int)(e % ld);
  const int j = (int)(e / ld);
  __bf16 h = (__bf16)0.f, l = (__bf16)0.f;
  if (i < ns && j < ns) {
    const double z = Z[i + (int64_t)j * ns];
    h = (__bf16)(float)z;
    l = (__bf16)(float)(z - (double)(float)h);
  }
  zh[e] = h;
  zl[e] = l;
}

// Lane (r32, g) of fragment f holds X[i][pcol[f]] for the 8 columns i = k0 + 16 s + 8 g + e
// of each 16-wide K step s; columns past ns are clamped (Z is zero there).
__device__ __forceinline__ void rot_load_x(float (&xv)[2][2][8], const float* __restrict__ X, int64_t nd, int ns,
                                           const int64_t (&pcol)[2], int k0, int g) {
#pragma unroll
  for (int s = 0; s < 2; ++s)
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int i = min(k0 + 16 * s + 8 * g + e, ns - 1);
      const float* row = X + (int64_t)i * nd;
#pragma unroll
      for (int f = 0; f < 2; ++f) xv[s][f][e] = row[pcol[f]];
    }
}

__device__ __forceinline__ void rot_load_z(u32x4 (&zr)[4], const __bf16* __restrict__ pzh,
                                           const __bf16* __restrict__ pzl, int k0) {
  zr[0] = *reinterpret_cast<const u32x4*>(pzh + k0);
  zr[1] = *reinterpret_cast<const u32x4*>(pzh + k0 + 8);
  zr[2] = *reinterpret_cast<const u32x4*>(pzl + k0);
  zr[3] = *reinterpret_cast<const u32x4*>(pzl + k0 + 8);
}

__device__ __forceinline__ void rot_store_z(const u32x4 (&zr)[4], __bf16* sh, __bf16* sl) {
  *reinterpret_cast<u32x4*>(sh) = zr[0];
  *reinterpret_cast<u32x4*>(sh + 8) = zr[1];
  *reinterpret_cast<u32x4*>(sl) = zr[2];
  *reinterpret_cast<u32x4*>(sl + 8) = zr[3];
}

__global__ __launch_bounds__(256) void rotate_bf16x3_kernel(const float* __restrict__ X, const __bf16* __restrict__ zh,
                                                            const __bf16* __restrict__ zl, float* __restrict__ O,
                                                            int64_t nd, int ns, int ld, int npt, int njt,
                                                            int per_xcd) {
  __shared__ __attribute__((aligned(16))) __bf16 lds[2][2][kRotJ * kLd];  // [buffer][hi, lo][j][kLd]
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  // blocks are dealt to the 8 XCDs round-robin; a contiguous run of logical tiles per
  // XCD keeps the njt blocks that read one slab of X on one L2
  const int b = blockIdx.x;
  const int logical = (b % 8) * per_xcd + b / 8;
  if (logical >= npt * njt) return;
  const int ptile = logical / njt, jtile = logical % njt;
  const int j0 = jtile * kRotJ;
  const int64_t p0 = (int64_t)ptile * kRotP + wave * 64;

  // Z staging: thread t copies 16 bf16 of column j0 + t / 2 (hi and lo)
  const int zrow = tid >> 1, zhalf = tid & 1;
  const __bf16* pzh = zh + (int64_t)(j0 + zrow) * ld + 16 * zhalf;
  const __bf16* pzl = zl + (int64_t)(j0 + zrow) * ld + 16 * zhalf;
  const int zoff = zrow * kLd + 16 * zhalf;

  // X gather: fragment f covers points p0 + 32 f + (lane % 32); K slot 8 (lane / 32) + e
  const int r32 = lane & 31, g = lane >> 5;
  int64_t pcol[2];
#pragma unroll
  for (int f = 0; f < 2; ++f) pcol[f] = min(p0 + 32 * f + r32, nd - 1);

  f32x16 acc[4][2];  // [j fragment][p fragment]
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int v = 0; v < 16; ++v) acc[i][j][v] = 0.f;

  const int nstage = ld / kKS;
  float xc[2][2][8];  // [k16 step][p fragment][e]
  u32x4 zr[4];
  rot_load_z(zr, pzh, pzl, 0);
  rot_load_x(xc, X, nd, ns, pcol, 0, g);
  rot_store_z(zr, lds[0][0] + zoff, lds[0][1] + zoff);
  __syncthreads();

  for (int t = 0; t < nstage; ++t) {
    const int buf = t & 1;
    const bool more = t + 1 < nstage;
    float xn[2][2][8];
    if (more) {
      rot_load_z(zr, pzh, pzl, (t + 1) * kKS);
      rot_load_x(xn, X, nd, ns, pcol, (t + 1) * kKS, g);
    }
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      bf16x8 xh[2], xl[2];
#pragma unroll
      for (int f = 0; f < 2; ++f) split8(xc[s][f], xh[f], xl[f]);
#pragma unroll
      for (int jf = 0; jf < 4; ++jf) {
        const int o = (jf * 32 + r32) * kLd + 16 * s + 8 * g;
        const bf16x8 zhv = as_bf8(*reinterpret_cast<const u32x4*>(lds[buf][0] + o));
        const bf16x8 zlv = as_bf8(*reinterpret_cast<const u32x4*>(lds[buf][1] + o));
#pragma unroll
        for (int f = 0; f < 2; ++f) acc[jf][f] = mfma_bf16(zlv, xh[f], acc[jf][f]);
#pragma unroll
        for (int f = 0; f < 2; ++f) acc[jf][f] = mfma_bf16(zhv, xl[f], acc[jf][f]);
#pragma unroll
        for (int f = 0; f < 2; ++f) acc[jf][f] = mfma_bf16(zhv, xh[f], acc[jf][f]);
      }
    }
    if (more) {
      rot_store_z(zr, lds[buf ^ 1][0] + zoff, lds[buf ^ 1][1] + zoff);
#pragma unroll
      for (int s = 0; s < 2; ++s)
#pragma unroll
        for (int f = 0; f < 2; ++f)
#pragma unroll
          for (int e = 0; e < 8; ++e) xc[s][f][e] = xn[s][f][e];
    }
    __syncthreads();
  }

  // D[j][p]: lane l, register v -> j = 8 (v / 4) + 4 (l / 32) + v % 4, p = l % 32
#pragma unroll
  for (int jf = 0; jf < 4; ++jf)
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      const int j = j0 + jf * 32 + 8 * (v >> 2) + 4 * g + (v & 3);
      if (j >= ns) continue;
#pragma unroll
      for (int f = 0; f < 2; ++f) {
        const int64_t p = p0 + 32 * f + r32;
        if (p < nd) O[(int64_t)j * nd + p] = acc[jf][f][v];
      }
    }
}

hipError_t launch_rotate_bf16x3(const float* X, const double* Z, void* zsplit, float* O, int64_t nd, int ns,
                                hipStream_t s) {
  const int ld = (int)zsplit_ld(ns);
  const int cols = (int)zsplit_cols(ns);
  __bf16* zh = static_cast<__bf16*>(zsplit);
  __bf16* zl = zh + (size_t)ld * cols;
  const int64_t nz = (int64_t)ld * cols;
  hipLaunchKernelGGL(zsplit_kernel, dim3((unsigned)((nz + 255) / 256)), dim3(256), 0, s, Z, ns, ld, cols, zh, zl);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int npt = (int)((nd + kRotP - 1) / kRotP);
  const int njt = cols / kRotJ;
  const int64_t nb = (int64_t)npt * njt;
  const int per_xcd = (int)((nb + 7) / 8);
  hipLaunchKernelGGL(rotate_bf16x3_kernel, dim3((unsigned)(per_xcd * 8)), dim3(256), 0, s, X, zh, zl, O, nd, ns, ld,
                     npt, njt, per_xcd);
  return hipGetLastError();
}

}  // namespace chefsi
