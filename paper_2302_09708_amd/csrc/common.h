// Internal declarations shared by the HIP kernels and the host runtime of libchefsi.
// Not part of the public ABI (that is include/chefsi.h).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace chefsi {

constexpr int kMaxRadius = 6;  // finite-difference order up to 12
constexpr int kVecThreads = 256;   // fixed-grid reductions (Lanczos sums, stress sums)
constexpr int kVecBlocks = 1024;
constexpr int kHxMaxThreads = 512;  // widest supported x row (one thread per x point)
// stencil threads per block for PY rows per thread (1024 keeps 128 VGPRs per lane, 512 keeps 256)
constexpr int hx_max_threads(int py) { return py == 1 ? 1024 : 512; }
constexpr int kHxMaxHalo = 4;            // halo values each stencil thread stages per plane
constexpr int kHxDummy = 64;             // per-lane dummy LDS slots after each stencil buffer
constexpr size_t kHxMaxLds = 96 * 1024;  // dynamic LDS of one stencil block (gfx950: 160 KB per CU)

// ---------------------------------------------------------------------------
// hx_apply: fused  out = sa * ((H_loc x) - sc * x) + sb * prev   for a block of vectors,
// H_loc x = c0 x + sum_p cx[p](x[i+-p ex]) + cy.. + cz.. + veff x + (projector term of the
// points whose record fits four entries; the rest of V_nl x is added by nl_scatter).
// TI: element type of x; TC: arithmetic type; TO: element type of prev/out.
// ---------------------------------------------------------------------------
template <typename TC>
struct alignas(16) HxRec {
  int lidx;     // point inside the tile plane: ly * nx + x
  int c01;      // alpha columns of entries 0 and 1 (16 bits each)
  int c23;      // alpha columns of entries 2 and 3
  int pad;
  TC val[4];    // chi values of the (up to) four entries, zero past the last
};

template <typename TI, typename TC, typename TO>
struct HxArgs {
  const TI* x;
  const TO* prev;  // may be null when sb == 0
  TO* out;
  const TC* veff;
  // projector term of the points with at most four entries (the others go to nl_scatter):
  // one record per point, grouped by (y tile, z plane); rec_ptr == null when there are none
  const int* rec_ptr;      // nty * nz + 1: records of (tile t, plane z) are [rec_ptr[t*nz+z], rec_ptr[t*nz+z+1])
  const HxRec<TC>* rec;
  const TC* alpha;         // ns x np_tot, projector column fastest (staged in LDS per block)
  int np_tot;
  int nx, ny, nz;
  int64_t nd;           // leading dimension of x, prev, out
  int per_x, per_y, per_z;  // 1 = periodic, 0 = Dirichlet
  TC c0;                    // centre weight: -1/2 w0 sum_d h_d^-2
  TC cx[kMaxRadius + 1], cy[kMaxRadius + 1], cz[kMaxRadius + 1];  // -1/2 w_p / h_d^2
  TC sa, sc, sb;
  // tiling
  int nyg;   // thread rows (y groups) per block; threads used = nx * nyg
  int ty;    // tile rows = nyg * PY
  int nty;   // tiles along y
  int zc;    // planes per z chunk
  int nzc;   // z chunks
  int64_t nblocks;  // nty * nzc * ns
  int per_xcd;      // blocks per XCD after padding the grid to a multiple of 8
  int pitch;        // LDS row pitch in elements (hx_pitch)
};

// LDS row pitch of the stencil tile: at least nx + 2r (the x halo).  A wave covers whole
// x rows of consecutive row groups, and the rows of neighbouring groups lie py rows apart,
// so the lanes of a wave that straddles two groups fall on distinct LDS banks when
// py * pitch = nx modulo the 256 bytes the banks span (each lane then reads the 8- or
// 4-byte slot after its predecessor's).  The smallest such pitch is taken; when none
// exists (py even and nx odd) nx plus a whole multiple of 256 bytes, which satisfies it
// for one row per thread.
__host__ __device__ inline int hx_pitch(int nx, int radius, int elem_bytes, int py) {
  const int g = 256 / elem_bytes;
  const int base = nx + 2 * radius;
  for (int p = base; p < base + g; ++p)
    if (((py * p - nx) % g + g) % g == 0) return p;
  return nx + ((2 * radius + g - 1) / g) * g;
}

struct HxPlan {
  bool ok = false;  // false: no tiling fits this grid
  int py = 2;
  int nyg = 1;
  int ty = 2;
  int nty = 1;
  int zc = 1;
  int nzc = 1;
  int threads = 64;
  int kh = 4;        // halo values each thread stages per plane (2, 3 or 4)
  size_t lds_tile_bytes = 0;  // two tile planes
};

// Choose the tiling for one grid (deterministic in the shape only; ns only sets the z chunks).
// py_override / nyg_override > 0 restrict the search to that rows-per-thread / row-group
// count (the result's ok is false when the restricted tiling does not fit).
HxPlan plan_hx(int nx, int ny, int nz, int ns, int radius, int elem_bytes, int py_override, int nyg_override);

// Dynamic LDS of one stencil block; np_tot < 0: no projector records.
size_t hx_lds_bytes(const HxPlan& p, int nx, int radius, int elem_bytes, int np_tot, int acc_bytes);

template <typename TI, typename TC, typename TO>
hipError_t launch_hx(const HxArgs<TI, TC, TO>& a, const HxPlan& p, int radius, int ns, hipStream_t s);

// ---------------------------------------------------------------------------
// nl_project: alpha[v * np_tot + q] = gdv[q] * sum_{s in S_J} chi_J[s, a] * y[v * nd + S_J[s]]
// for every atom J, projector a (q = poff[J] + a) and vector v.
// ---------------------------------------------------------------------------
template <typename TI, typename TC>
struct NlArgs {
  const TI* y;
  int64_t nd;
  int ns;
  int n_atoms;
  const int* supp_off;  // n_atoms + 1, offsets into supp_idx
  const int* supp_idx;
  const int64_t* chi_off;  // n_atoms, offset of chi_J
  const int* nproj;        // n_atoms
  const int* poff;         // n_atoms, first projector column of atom J
  const TC* chi;
  const TC* gdv;           // gamma * dV per projector column
  TC* alpha;
  int np_tot;
  int ngroups;  // orbital groups per atom (set by the launcher)
  int per_xcd;  // blocks per XCD (set by the launcher)
};

template <typename TI, typename TC>
hipError_t launch_nl_project(const NlArgs<TI, TC>& a, hipStream_t s);

// ---------------------------------------------------------------------------
// nl_scatter: out[v * nd + p] += sa * sum_{e in entries of p} val[e] * alpha[v * np_tot + col[e]]
// for every support point p (one record per point: {p, first entry, entry count, 0},
// entries padded to a multiple of four) and vector v.
// ---------------------------------------------------------------------------
template <typename TC, typename TO>
struct NsArgs {
  TO* out;
  int64_t nd;
  int ns;
  const int4* rec;
  int n_pts;
  const int* col;
  const TC* val;
  const TC* alpha;
  int np_tot;
  TC sa;
};

template <typename TC, typename TO>
hipError_t launch_nl_scatter(const NsArgs<TC, TO>& a, hipStream_t s);

// ---------------------------------------------------------------------------
// nl_band: the whole projector term of H y in one pass over the touched points, region by
// region (a region = a run of consecutive touched points in grid index order, packed up to
// kBandMaxPts points, kBandMaxSlots projectors and kBandMaxEnt projector entries).
// A block owns one region and a run of orbital groups of G orbitals; it stages the
// region's entry tables in LDS once and, group by group:
//   scatter (optional): y[v][i] += sa * sum_{e in entries(i)} chi_e * alpha[q_e][v], written
//   in place (alpha projector-major: alpha[q * ns + v]);
//   gather: for every projector q touching the region (a slot), partial[slot][v] =
//   sum over the region's points of q, in index order, of chi * y[v][i] (the final y);
// and nl_band_reduce forms alpha[q][v] = gdv[q] * sum of q's slots in region order.  Every
// sum has a fixed order: the result does not depend on scheduling.
// ---------------------------------------------------------------------------
constexpr int kBandThreads = 512;   // one thread per point of the region
constexpr int kBandMaxPts = 512;    // touched points of one region (LDS: kBandMaxPts * G values)
constexpr int kBandMaxSlots = 128;  // projectors touching one region (their coefficients staged in LDS)
constexpr int kBandMaxEnt = 1920;   // projector entries of one region (scatter and gather tables in LDS)

template <typename TY, typename TC>
struct NbArgs {
  TY* y;               // Nd x ns block (ld nd): scattered in place when scatter, read otherwise
  int64_t nd;
  int ns;
  int nreg;
  const int* reg_pt;   // nreg + 1: points of region r are [reg_pt[r], reg_pt[r + 1])
  const int* pt_idx;   // grid index of each point
  const int* pt_ent;   // npts + 1: entries of point p
  const int* ent_ls;   // region slot of each entry (the projector's place among the region's slots)
  const TC* ent_chi;
  const int* reg_slot;  // nreg + 1: slots of region r
  const int* slot_q;    // projector column of each slot
  const int* slot_ent;  // nslots + 1: gather entries of slot s
  const int* gent_loc;  // point of each gather entry, relative to its region's first point
  const TC* gent_chi;
  const TC* alpha;      // scatter: projector-major coefficients (the region's staged in LDS)
  TC sa;
  TC* partial;          // nslots x ns, projector slot major
  int ngroups;          // orbital groups (set by the launcher)
  int gpc;              // orbital groups per block (set by the launcher)
  int nchunks;          // blocks per region (set by the launcher)
  int per_xcd;          // blocks per XCD (set by the launcher)
};

template <typename TY, typename TC>
hipError_t launch_nl_band(const NbArgs<TY, TC>& a, bool scatter, bool gather, hipStream_t s);
template <typename TC>
hipError_t launch_nl_band_reduce(const TC* partial, const int* q_slot_ptr, const int* q_slot, const TC* gdv,
                                 int np_tot, int ns, TC* alpha, hipStream_t s);

// ---------------------------------------------------------------------------
// Dense products on MFMA.
// gram:   partial[split][tile] = A(:, I)^T B(:, J) over a K range, for upper tiles I <= J.
// reduce: C(i, j) = C(j, i) = sum_split partial (i <= j), C is ns x ns, ld ns, FP64.
// rotate: O = X Z  (X: nd x ns, ld nd; Z: ns x ns, ld ns; O: nd x ns, ld nd).
// ---------------------------------------------------------------------------
struct GramPlan {
  int tile = 128;
  int nt = 1;        // tiles per dimension
  int ntiles = 1;    // upper tiles nt (nt + 1) / 2
  int splits = 1;
  int64_t kchunk = 0;
  size_t partial_bytes = 0;
};

GramPlan plan_gram(int64_t nd, int ns);

template <typename TA, typename TB>
hipError_t launch_gram_f64(const TA* A, const TB* B, int64_t nd, int ns, const GramPlan& p, double* partial,
                           hipStream_t s);

hipError_t launch_gram_reduce(const double* partial, const GramPlan& p, int ns, double* C, hipStream_t s);

// C(i, j) = C(j, i) = sum over the nparts column-major ns x ns partial products P (upper
// triangle read, summed in a fixed order).
hipError_t launch_sum_partials(const double* P, int nparts, int ns, double* C, hipStream_t s);

// Row panels of an FP32 block for the FP64 library products of a mixed handle's
// refinement: W(i, c) = double(X(i, c)) and O(i, c) = float(P(i, c)), i < r, c < ns
// (X, O: ld ldx; W, P: ld ldw).
hipError_t launch_widen_rows(const float* X, int64_t ldx, int64_t r, int ns, double* W, int64_t ldw,
                             hipStream_t s);
hipError_t launch_narrow_rows(const double* P, int64_t ldw, int64_t r, int ns, float* O, int64_t ldx,
                              hipStream_t s);

// Diagonal scaling of the pencil (Hs, Ms) by sc_i = Ms_ii^-1/2 (sc: ns doubles, written),
// and the matching back-transformation Z(i, j) <- sc_i Z(i, j).
hipError_t launch_pencil_scale(double* Hs, double* Ms, double* sc, int ns, hipStream_t s);
hipError_t launch_row_scale(double* Z, const double* sc, int ns, hipStream_t s);
// d[i] = A(i, i) for an ns x ns column-major matrix
hipError_t launch_copy_diag(const double* A, double* d, int ns, hipStream_t s);

template <typename TX, typename TO>
hipError_t launch_rotate_f64(const TX* X, const double* Z, TO* O, int64_t nd, int ns, hipStream_t s);

// Split-bf16 variants for FP32 blocks (three bf16 MFMAs per product, FP32 accumulation).
// gram: same plan, partial layout and reduction as the FP64 kernel.
// rotate: Z (FP64) is first split into the zsplit scratch (zsplit_bytes(ns) bytes).
hipError_t launch_gram_bf16x3(const float* A, const float* B, int64_t nd, int ns, const GramPlan& p,
                              double* partial, hipStream_t s);
size_t zsplit_bytes(int ns);
hipError_t launch_rotate_bf16x3(const float* X, const double* Z, void* zsplit, float* O, int64_t nd, int ns,
                                hipStream_t s);

// ---------------------------------------------------------------------------
// Nonlocal forces: out = d x / d x_dir (central FD, c[1..r], periodic or zero ghosts),
// then forces[J*3 + dir] = -2 sum_k (gdv[q]/dv) sum_v occ[v] alpha[v*np+q] beta[v*np+q].
// ---------------------------------------------------------------------------
template <typename TV>
struct GradArgs {
  const TV* x;
  double* out;
  int64_t nd;
  int nx, ny, nz;
  int dir, r, periodic;
  double c[kMaxRadius + 1];
  double inv_h;
};

struct ForceArgs {
  const double* alpha;
  const double* beta;
  const double* occ;
  const double* gdv;
  const int* nproj;
  const int* poff;
  double dv;
  int n_atoms, np_tot, ns, dir;
  double* forces;
};

template <typename TV>
hipError_t launch_grad(const GradArgs<TV>& a, int ns, hipStream_t s);

// Kinetic stress sums: out[0..5] = sum_v occ[v] sum_i g_a g_b for ab = xx, yy, zz, xy, xz,
// yz (g = FD gradient of orbital v); partial: kVecBlocks * 6 doubles of scratch.
template <typename TV>
struct StressArgs {
  const TV* x;
  const double* occ;
  int64_t nd;
  int ns;
  int nx, ny, nz, r;
  int periodic[3];
  double c[kMaxRadius + 1];
  double inv_h[3];
  double* partial;
  double* out;
};

template <typename TV>
hipError_t launch_stress_sums(const StressArgs<TV>& a, hipStream_t s);
// Nonlocal stress weights: out[b * nchi + e] = chi[e] * disp[3 s + b] (b = 0..2) for every
// projector value e (atom-major, the layout of chi) at its support point s.
struct ChiDispArgs {
  const double* chi;
  const double* disp;     // 3 per support point, support-point order of supp_idx
  const int* supp_off;    // n_atoms + 1
  const int64_t* chi_off; // n_atoms
  const int* nproj;       // n_atoms
  int n_atoms;
  int64_t nchi;
  double* out;            // 3 * nchi
};
hipError_t launch_chi_disp(const ChiDispArgs& a, hipStream_t s);
hipError_t launch_forces(const ForceArgs& a, hipStream_t s);

// ---------------------------------------------------------------------------
// Lanczos vector kernels (fixed grid of kVecBlocks x kVecThreads, fixed-order sums).
// dot:   w -= beta vp (vp may be null); out[0] = v . w
// norm:  w -= alpha v (v may be null);  out[0] = w . w
// scale: out = TV(w * inv);  widen: w = double(x)
// partial: kVecBlocks doubles of scratch.
// ---------------------------------------------------------------------------

template <typename TV>
hipError_t launch_lanczos_dot(double* w, const TV* v, const TV* vp, double beta, int64_t n, double* partial,
                              double* out, hipStream_t s);
template <typename TV>
hipError_t launch_lanczos_norm(double* w, const TV* v, double alpha, int64_t n, double* partial, double* out,
                               hipStream_t s);
template <typename TV>
hipError_t launch_lanczos_scale(const double* w, double inv, int64_t n, TV* out, hipStream_t s);
template <typename TV>
hipError_t launch_widen(const TV* x, int64_t n, double* w, hipStream_t s);

// ---------------------------------------------------------------------------
// H at a Bloch wavevector on complex FP64 blocks (interleaved re/im, Nd x Ns, ld Nd).
// ---------------------------------------------------------------------------
struct ZHxArgs {
  const double2* x;
  const double2* prev;  // may be null (sb unused)
  double2* out;
  const double* veff;
  int n[3];
  int per[3];       // 1 = periodic (Bloch-phased ghosts), 0 = Dirichlet (zero ghosts)
  int r;
  int64_t nd;
  double c0;                     // -1/2 w0 sum_d h_d^-2
  double cw[3][kMaxRadius + 1];  // -1/2 w_p / h_d^2
  double2 ph[3];                 // exp(i k_d L_d)
  double sa, sc, sb;
};

// tiling of the complex stencil pass (one row of a tile per thread)
constexpr int kZMaxThreads = 512;
struct ZTiling {
  int ty, nty, zc, nzc, threads, pitch, kh;
  size_t lds_bytes;
  int64_t nblocks;
  int per_xcd;
};
ZTiling plan_zhx(int nx, int ny, int nz, int ns, int radius);

// complex band pass (the real band pass's regions and tables with chi~ values; the gather
// table holds conj(chi~)); alpha projector-major: alpha[q * ns + v]
constexpr int kZBandMaxEnt = 1024;  // projector entries of one region (complex tables in LDS)
struct ZNbArgs {
  double2* y;  // Nd x ns block (ld nd): scattered in place when scatter, read otherwise
  int64_t nd;
  int ns;
  int nreg;
  const int* reg_pt;
  const int* pt_idx;
  const int* pt_ent;
  const int* ent_ls;
  const double2* ent_chi;
  const int* reg_slot;
  const int* slot_q;
  const int* slot_ent;
  const int* gent_loc;
  const double2* gent_chi;
  const double2* alpha;
  double sa;
  double2* partial;  // nslots x ns, slot major
  int ngroups, gpc, nchunks, per_xcd;  // set by the launcher
};

hipError_t launch_zhx(const ZHxArgs& a, int ns, hipStream_t s);
hipError_t launch_zband(const ZNbArgs& a, bool scatter, bool gather, hipStream_t s);
hipError_t launch_zband_reduce(const double2* partial, const int* q_slot_ptr, const int* q_slot, const double* gdv,
                               int np_tot, int ns, double2* alpha, hipStream_t s);
// C = Hermitian completion of sum_q P_q (upper triangles read, fixed order), P: nparts
// column-major ns x ns complex partial products.
hipError_t launch_zsum_partials(const double2* P, int nparts, int ns, double2* C, hipStream_t s);

}  // namespace chefsi
