// Dense contractions of the projection and rotation steps on FP64 MFMA (gfx950).
//
// Projection (Alg. 1; Sec. 2.2):  Hs = X~^T Y~ and Ms = X~^T X~, an (Nd x Ns)^T (Nd x Ns)
//   product with K = Nd in the hundreds of thousands.  The paper forms row-block
//   partial products on each GPU and sums them; here the same split of K runs as
//   split-K inside one GPU: every block owns one 128 x 128 output tile of the upper
//   triangle (both results are symmetric) over one K chunk, writes its partial
//   tile, and a second kernel sums the partials in a fixed order and mirrors the
//   upper triangle (deterministic, no atomics).
// Rotation (Alg. 1; Sec. 2.4):  X = X~ Z~, (Nd x Ns)(Ns x Ns).
//
// v_mfma_f64_16x16x4f64 lane layout (measured): operand A[i][k] comes from lane
// i + 16k, B[k][j] from lane j + 16k, and result D[i][j] lands in lane
// j + 16 (i % 4), register i / 4.  Because a contraction may visit K in any order,
// lane group g = lane / 16 takes the four consecutive k = 4g .. 4g+3 of each
// 16-wide K step, one per MFMA, so every lane loads 32 contiguous bytes of a column.
#include "common.h"

#include <algorithm>

namespace chefsi {

typedef double d4 __attribute__((ext_vector_type(4)));

constexpr int kTile = 128;  // block tile (both dimensions)
constexpr int kFr = 4;      // 16 x 16 fragments per wave along each dimension (wave tile 64 x 64)

__device__ __forceinline__ d4 mfma_f64(double a, double b, d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// (ti, tj) of upper tile t in row-major order of the upper triangle of an nt x nt tile grid.
__device__ __forceinline__ void upper_tile(int t, int nt, int& ti, int& tj) {
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

template <typename TA, typename TB>
__global__ __launch_bounds__(256) void gram_f64_kernel(const TA* __restrict__ A, const TB* __restrict__ B, int64_t nd,
                                                       int ns, int nt, int ntiles, int64_t kchunk,
                                                       double* __restrict__ partial) {
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int wm = wave & 1, wn = wave >> 1;
  const int g = lane >> 4, r = lane & 15;
  const int tile = blockIdx.x % ntiles;
  const int split = blockIdx.x / ntiles;
  int ti, tj;
  upper_tile(tile, nt, ti, tj);
  const int64_t kb = (int64_t)split * kchunk;
  const int64_t ke = min(nd, kb + kchunk);

  const TA* pa[kFr];
  const TB* pb[kFr];
#pragma unroll
  for (int f = 0; f < kFr; ++f) {
    const int ci = min(ti * kTile + wm * 64 + f * 16 + r, ns - 1);
    const int cj = min(tj * kTile + wn * 64 + f * 16 + r, ns - 1);
    pa[f] = A + (int64_t)ci * nd + 4 * g;
    pb[f] = B + (int64_t)cj * nd + 4 * g;
  }

  d4 acc[kFr][kFr];
#pragma unroll
  for (int i = 0; i < kFr; ++i)
#pragma unroll
    for (int j = 0; j < kFr; ++j) acc[i][j] = d4{0.0, 0.0, 0.0, 0.0};

  double av[kFr][4], bv[kFr][4];
  const int64_t kfull = kb + ((ke - kb) / 16) * 16;
  int64_t k = kb;
  if (k < kfull) {
#pragma unroll
    for (int f = 0; f < kFr; ++f)
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        av[f][s] = double(pa[f][k + s]);
        bv[f][s] = double(pb[f][k + s]);
      }
  }
  for (; k < kfull; k += 16) {
    double an[kFr][4], bn[kFr][4];
    const bool more = k + 16 < kfull;
#pragma unroll
    for (int f = 0; f < kFr; ++f)
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        an[f][s] = more ? double(pa[f][k + 16 + s]) : 0.0;
        bn[f][s] = more ? double(pb[f][k + 16 + s]) : 0.0;
      }
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
      for (int i = 0; i < kFr; ++i)
#pragma unroll
        for (int j = 0; j < kFr; ++j) acc[i][j] = mfma_f64(av[i][s], bv[j][s], acc[i][j]);
#pragma unroll
    for (int f = 0; f < kFr; ++f)
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        av[f][s] = an[f][s];
        bv[f][s] = bn[f][s];
      }
  }
  if (kfull < ke) {  // ragged K tail
#pragma unroll
    for (int f = 0; f < kFr; ++f)
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        const int64_t kk = kfull + 4 * g + s;
        av[f][s] = kk < ke ? double(pa[f][kfull + s]) : 0.0;
        bv[f][s] = kk < ke ? double(pb[f][kfull + s]) : 0.0;
      }
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
      for (int i = 0; i < kFr; ++i)
#pragma unroll
        for (int j = 0; j < kFr; ++j) acc[i][j] = mfma_f64(av[i][s], bv[j][s], acc[i][j]);
  }

  // partial tile, row-major 128 x 128: element (ii, jj) at ii * 128 + jj
  double* pt = partial + ((int64_t)split * ntiles + tile) * (kTile * kTile);
#pragma unroll
  for (int i = 0; i < kFr; ++i)
#pragma unroll
    for (int j = 0; j < kFr; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int ii = wm * 64 + i * 16 + g + 4 * v;
        const int jj = wn * 64 + j * 16 + r;
        pt[ii * kTile + jj] = acc[i][j][v];
      }
}

__global__ __launch_bounds__(256) void gram_reduce_kernel(const double* __restrict__ partial, int ns, int nt,
                                                          int ntiles, int splits, double* __restrict__ C) {
  const int tile = blockIdx.y;
  const int e = blockIdx.x * 256 + threadIdx.x;
  if (e >= kTile * kTile) return;
  int ti, tj;
  upper_tile(tile, nt, ti, tj);
  const int ii = e / kTile, jj = e % kTile;
  const int i = ti * kTile + ii, j = tj * kTile + jj;
  if (i >= ns || j >= ns || i > j) return;
  double sum = 0.0;
  const int64_t stride = (int64_t)ntiles * kTile * kTile;
  const double* p = partial + (int64_t)tile * kTile * kTile + e;
  for (int s = 0; s < splits; ++s) sum += p[s * stride];
  C[(int64_t)i + (int64_t)j * ns] = sum;
  C[(int64_t)j + (int64_t)i * ns] = sum;
}

// C(i, j) = C(j, i) = sum_p P_p(i, j) for i <= j, P_p column-major ns x ns, summed in p order.
__global__ __launch_bounds__(256) void sum_partials_kernel(const double* __restrict__ P, int nparts, int ns,
                                                           double* __restrict__ C) {
  const int64_t n2 = (int64_t)ns * ns;
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= n2) return;
  const int j = (int)(e / ns), i = (int)(e % ns);
  if (i > j) return;
  double sum = 0.0;
  for (int q = 0; q < nparts; ++q) sum += P[q * n2 + e];
  C[e] = sum;
  C[(int64_t)i * ns + j] = sum;
}

hipError_t launch_sum_partials(const double* P, int nparts, int ns, double* C, hipStream_t s) {
  const int64_t n2 = (int64_t)ns * ns;
  hipLaunchKernelGGL(sum_partials_kernel, dim3((unsigned)((n2 + 255) / 256)), dim3(256), 0, s, P, nparts, ns, C);
  return hipGetLastError();
}

// Row panels of an FP32 block for FP64 library products: W(i, c) = double(X(i, c)) and
// O(i, c) = float(P(i, c)) for i < r, c < ns (X, O: ld ldx; W, P: ld ldw).  Columns are
// dealt over grid.y, rows over grid.x; the FP64 -> FP32 step rounds to nearest.
__global__ __launch_bounds__(256) void widen_rows_kernel(const float* __restrict__ X, int64_t ldx, int64_t r,
                                                         int ns, double* __restrict__ W, int64_t ldw) {
  for (int c = blockIdx.y; c < ns; c += gridDim.y)
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < r; i += (int64_t)gridDim.x * 256)
      W[c * ldw + i] = double(X[c * ldx + i]);
}

__global__ __launch_bounds__(256) void narrow_rows_kernel(const double* __restrict__ P, int64_t ldw, int64_t r,
                                                          int ns, float* __restrict__ O, int64_t ldx) {
  for (int c = blockIdx.y; c < ns; c += gridDim.y)
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < r; i += (int64_t)gridDim.x * 256)
      O[c * ldx + i] = float(P[c * ldw + i]);
}

namespace {
dim3 panel_grid(int64_t r, int ns) {
  const int64_t bx = std::min<int64_t>((r + 255) / 256, 64);
  return dim3((unsigned)std::max<int64_t>(bx, 1), (unsigned)std::min(std::max(ns, 1), 1024));
}
}  // namespace

hipError_t launch_widen_rows(const float* X, int64_t ldx, int64_t r, int ns, double* W, int64_t ldw,
                             hipStream_t s) {
  if (r <= 0 || ns <= 0) return hipSuccess;
  hipLaunchKernelGGL(widen_rows_kernel, panel_grid(r, ns), dim3(256), 0, s, X, ldx, r, ns, W, ldw);
  return hipGetLastError();
}

hipError_t launch_narrow_rows(const double* P, int64_t ldw, int64_t r, int ns, float* O, int64_t ldx,
                              hipStream_t s) {
  if (r <= 0 || ns <= 0) return hipSuccess;
  hipLaunchKernelGGL(narrow_rows_kernel, panel_grid(r, ns), dim3(256), 0, s, P, ldw, r, ns, O, ldx);
  return hipGetLastError();
}

GramPlan plan_gram(int64_t nd, int ns) {
  GramPlan p;
  p.tile = kTile;
  p.nt = (ns + kTile - 1) / kTile;
  p.ntiles = p.nt * (p.nt + 1) / 2;
  // aim at ~1024 blocks (4 per CU), K chunks of at least 2048
  int splits = std::max(1, (1024 + p.ntiles - 1) / p.ntiles);
  const int64_t max_splits = std::max<int64_t>(1, nd / 2048);
  splits = (int)std::min<int64_t>(splits, max_splits);
  int64_t kchunk = (nd + splits - 1) / splits;
  kchunk = (kchunk + 15) / 16 * 16;
  splits = (int)((nd + kchunk - 1) / kchunk);
  p.splits = std::max(1, splits);
  p.kchunk = kchunk;
  p.partial_bytes = (size_t)p.splits * p.ntiles * kTile * kTile * sizeof(double);
  return p;
}

template <typename TA, typename TB>
hipError_t launch_gram_f64(const TA* A, const TB* B, int64_t nd, int ns, const GramPlan& p, double* partial,
                           hipStream_t s) {
  dim3 grid((unsigned)(p.ntiles * p.splits));
  hipLaunchKernelGGL((gram_f64_kernel<TA, TB>), grid, dim3(256), 0, s, A, B, nd, ns, p.nt, p.ntiles, p.kchunk,
                     partial);
  return hipGetLastError();
}

hipError_t launch_gram_reduce(const double* partial, const GramPlan& p, int ns, double* C, hipStream_t s) {
  dim3 grid((kTile * kTile + 255) / 256, (unsigned)p.ntiles);
  hipLaunchKernelGGL(gram_reduce_kernel, grid, dim3(256), 0, s, partial, ns, p.nt, p.ntiles, p.splits, C);
  return hipGetLastError();
}

// Symmetric diagonal scaling of the pencil before its Cholesky: s_i = Ms_ii^-1/2 (or 1
// when Ms_ii is not positive, so the Cholesky reports the failure), Hs <- S Hs S,
// Ms <- S Ms S.  The eigenvalues do not change; the eigenvectors of the scaled pencil
// map back as Z = S Z'.  It removes the spread of column norms that the filter leaves
// in the block, which otherwise limits the Cholesky in reduced precision.
__global__ void pencil_scale_kernel(double* __restrict__ Hs, double* __restrict__ Ms, const double* __restrict__ sc,
                                    int ns) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)ns * ns) return;
  const int i = (int)(e % ns), j = (int)(e / ns);
  const double f = sc[i] * sc[j];
  Hs[e] *= f;
  Ms[e] *= f;
}

__global__ void pencil_diag_kernel(const double* __restrict__ Ms, double* __restrict__ sc, int ns) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= ns) return;
  const double d = Ms[(int64_t)i * ns + i];
  sc[i] = d > 0.0 ? 1.0 / sqrt(d) : 1.0;
}

// Z(i, j) <- sc_i Z(i, j)
__global__ void row_scale_kernel(double* __restrict__ Z, const double* __restrict__ sc, int ns) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)ns * ns) return;
  Z[e] *= sc[(int)(e % ns)];
}

hipError_t launch_pencil_scale(double* Hs, double* Ms, double* sc, int ns, hipStream_t s) {
  hipLaunchKernelGGL(pencil_diag_kernel, dim3((unsigned)((ns + 255) / 256)), dim3(256), 0, s, Ms, sc, ns);
  const int64_t n2 = (int64_t)ns * ns;
  hipLaunchKernelGGL(pencil_scale_kernel, dim3((unsigned)((n2 + 255) / 256)), dim3(256), 0, s, Hs, Ms, sc, ns);
  return hipGetLastError();
}

__global__ void copy_diag_kernel(const double* __restrict__ A, double* __restrict__ d, int ns) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < ns) d[i] = A[(int64_t)i * ns + i];
}

hipError_t launch_copy_diag(const double* A, double* d, int ns, hipStream_t s) {
  hipLaunchKernelGGL(copy_diag_kernel, dim3((unsigned)((ns + 255) / 256)), dim3(256), 0, s, A, d, ns);
  return hipGetLastError();
}

hipError_t launch_row_scale(double* Z, const double* sc, int ns, hipStream_t s) {
  const int64_t n2 = (int64_t)ns * ns;
  hipLaunchKernelGGL(row_scale_kernel, dim3((unsigned)((n2 + 255) / 256)), dim3(256), 0, s, Z, sc, ns);
  return hipGetLastError();
}

// O = X Z computed as (Z^T X^T)^T so that the MFMA result rows run along the grid
// index m: each store writes 16 consecutive m (128 bytes) of 4 columns.
template <typename TX, typename TO>
__global__ __launch_bounds__(256) void rotate_f64_kernel(const TX* __restrict__ X, const double* __restrict__ Z,
                                                         TO* __restrict__ O, int64_t nd, int ns, int nmt, int nnt,
                                                         int per_xcd) {
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int wm = wave & 1, wn = wave >> 1;
  const int g = lane >> 4, r = lane & 15;
  // blocks are dealt to the 8 XCDs round-robin; give each XCD a contiguous run of
  // logical tiles so that the nnt blocks sharing one m panel of X share an L2
  const int b = blockIdx.x;
  const int logical = (b % 8) * per_xcd + b / 8;
  if (logical >= nmt * nnt) return;
  const int mt = logical / nnt, nt = logical % nnt;
  const int64_t m0 = (int64_t)mt * kTile + wm * 64;
  const int n0 = nt * kTile + wn * 64;

  const TX* px[kFr];     // X rows m for fragment f (column offset added per k)
  const double* pz[kFr]; // Z column n for fragment f
  bool mok[kFr], nok[kFr];
#pragma unroll
  for (int f = 0; f < kFr; ++f) {
    const int64_t m = m0 + f * 16 + r;
    mok[f] = m < nd;
    px[f] = X + (mok[f] ? m : 0);
    const int n = n0 + f * 16 + r;
    nok[f] = n < ns;
    pz[f] = Z + (int64_t)(nok[f] ? n : 0) * ns + 4 * g;
  }

  d4 acc[kFr][kFr];  // [n fragment][m fragment]
#pragma unroll
  for (int i = 0; i < kFr; ++i)
#pragma unroll
    for (int j = 0; j < kFr; ++j) acc[i][j] = d4{0.0, 0.0, 0.0, 0.0};

  for (int k = 0; k < ns; k += 16) {
    double zv[kFr][4], xv[kFr][4];
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const int kk = k + 4 * g + s;
      const bool kok = kk < ns;
      const int64_t col = (int64_t)(kok ? kk : 0) * nd;
#pragma unroll
      for (int f = 0; f < kFr; ++f) {
        zv[f][s] = kok ? pz[f][k + s] : 0.0;
        xv[f][s] = double(px[f][col]);
      }
    }
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
      for (int i = 0; i < kFr; ++i)
#pragma unroll
        for (int j = 0; j < kFr; ++j) acc[i][j] = mfma_f64(zv[i][s], xv[j][s], acc[i][j]);
  }

#pragma unroll
  for (int i = 0; i < kFr; ++i)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int n = n0 + i * 16 + g + 4 * v;
      if (n >= ns) continue;
#pragma unroll
      for (int j = 0; j < kFr; ++j) {
        if (!mok[j]) continue;
        const int64_t m = m0 + j * 16 + r;
        O[m + (int64_t)n * nd] = TO(acc[i][j][v]);
      }
    }
}

template <typename TX, typename TO>
hipError_t launch_rotate_f64(const TX* X, const double* Z, TO* O, int64_t nd, int ns, hipStream_t s) {
  const int nmt = (int)((nd + kTile - 1) / kTile);
  const int nnt = (ns + kTile - 1) / kTile;
  const int64_t nb = (int64_t)nmt * nnt;
  const int per_xcd = (int)((nb + 7) / 8);
  dim3 grid((unsigned)(per_xcd * 8));
  hipLaunchKernelGGL((rotate_f64_kernel<TX, TO>), grid, dim3(256), 0, s, X, Z, O, nd, ns, nmt, nnt, per_xcd);
  return hipGetLastError();
}

template hipError_t launch_gram_f64<double, double>(const double*, const double*, int64_t, int, const GramPlan&,
                                                    double*, hipStream_t);
template hipError_t launch_gram_f64<float, double>(const float*, const double*, int64_t, int, const GramPlan&,
                                                   double*, hipStream_t);
template hipError_t launch_gram_f64<float, float>(const float*, const float*, int64_t, int, const GramPlan&,
                                                  double*, hipStream_t);
template hipError_t launch_rotate_f64<double, double>(const double*, const double*, double*, int64_t, int,
                                                      hipStream_t);
template hipError_t launch_rotate_f64<float, float>(const float*, const double*, float*, int64_t, int, hipStream_t);

}  // namespace chefsi
