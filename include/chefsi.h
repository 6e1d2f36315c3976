/*
 * chefsi.h -- C-ABI of libchefsi.so: one Chebyshev-filtered subspace iteration
 * (CheFSI) step of real-space Kohn-Sham DFT on an AMD Instinct MI355X (gfx950).
 *
 * The operation is Algorithm 1 of Sharma et al., "GPU acceleration of local and
 * semilocal density functional calculations in the SPARC electronic structure
 * code" (arXiv:2302.09708):
 *
 *   Filtering        X~ = p_m((H - cI)/e) X,  c = (lam_hi + lam_cut)/2,
 *                    e = (lam_hi - lam_cut)/2                  (Alg. 1; Sec. 2.1)
 *   Projection       H~ = X~^T (H X~),  M~ = X~^T X~           (Alg. 1; Sec. 2.2)
 *   Diagonalization  H~ Z~ = M~ Z~ D~                           (Alg. 1; Sec. 2.3)
 *   Rotation         X = X~ Z~                                  (Alg. 1; Sec. 2.4)
 *
 * for the matrix-free Hamiltonian of Sec. 2.1,
 *
 *   H = -1/2 Lap_FD + diag(Veff) + sum_J chi_J diag(gamma_J) chi_J^T dV,
 *
 * with a central finite-difference Laplacian of even order n0 = 2r on a uniform
 * grid, periodic or Dirichlet per direction, and Kleinman-Bylander projectors
 * chi_J on the grid points S_J of atom J.  dV = hx*hy*hz.
 *
 * The filter is evaluated in its scaled three-term form: the result equals the
 * paper's p_m((H - cI)/e) X divided by the scalar p_m((lam_lo - c)/e), which
 * leaves every Ritz pair unchanged and keeps the iterates O(1).  "degree" m is
 * the number of H applications inside the filter; one more gives H X~.
 *
 * Conventions shared by every call
 *   - Grid point (x, y, z) has linear index i = x + Nx*(y + Ny*z).
 *   - An orbital block X is Nd x ns, column-major with leading dimension Nd
 *     (a row-major (ns, Nd) array whose row j is orbital j), in DEVICE memory.
 *     Its element type is double for CHEFSI_FP64 handles and float for
 *     CHEFSI_MIXED handles.
 *   - `ws` is caller-owned DEVICE memory of at least chefsi_workspace_bytes()
 *     bytes, 256-byte aligned.  Its contents on entry are ignored and on exit
 *     are unspecified.
 *   - `stream` is a hipStream_t (NULL = the null stream).  Every call enqueues
 *     its work on that stream; calls that return host data (Ritz values)
 *     synchronize the stream before returning.
 *   - Every call returns a chefsi_status (0 = CHEFSI_OK).  No exception or
 *     abort crosses the ABI.  After an error the handle stays valid, device
 *     outputs are unspecified and nothing leaks.
 *   - Handles are independent and thread-compatible (one handle per thread or
 *     per request); calls on one handle must not overlap.
 */
#ifndef CHEFSI_H
#define CHEFSI_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  CHEFSI_OK = 0,
  CHEFSI_ERR_INVALID_ARG = 1,  /* bad dims/order/bc, ns out of range, bad pointer, bad bounds     */
  CHEFSI_ERR_HIP = 2,          /* a HIP runtime call failed (message in chefsi_last_error)        */
  CHEFSI_ERR_WORKSPACE = 3,    /* ws_bytes smaller than chefsi_workspace_bytes()                   */
  CHEFSI_ERR_NOT_POSDEF = 4,   /* Cholesky of M~ failed: filtered block is numerically rank deficient */
  CHEFSI_ERR_EIG = 5,          /* dense eigensolver did not converge                               */
  CHEFSI_ERR_NONFINITE = 6,    /* NaN/Inf among the Ritz values                                    */
  CHEFSI_ERR_SOLVER = 7,       /* rocBLAS/rocSOLVER returned an error status                       */
  CHEFSI_ERR_OOM = 8           /* a library-internal allocation failed (create only)               */
} chefsi_status;

/* Arithmetic of a handle's steps (the dense eigensolve is FP64 in both):
 *   CHEFSI_FP64   X in double; filter, projection and rotation in FP64 (FP64 MFMA).
 *   CHEFSI_MIXED  X in float; filter in FP32; projection and rotation as split
 *                 bf16 products on MFMA (each FP32 value as hi + lo bf16, three
 *                 bf16 products, FP32 accumulation; Hs and Ms summed in FP64
 *                 over K chunks); Cholesky, eigensolve and chefsi_refine_fp64
 *                 in FP64. */
typedef enum { CHEFSI_FP64 = 0, CHEFSI_MIXED = 1 } chefsi_precision;

typedef struct chefsi_handle chefsi_handle_t;

/* Uniform grid (Sec. 2.1; the grid spacing is the method's single
 * discretisation parameter).  n[d] >= 1; in a periodic direction n[d] >= r
 * (r = fd_order/2).  fd_order even, 2..12.  h[d] > 0 (bohr). */
typedef struct {
  int32_t n[3];
  double h[3];
  int32_t bc[3];     /* 0 = periodic, 1 = Dirichlet (zero outside nodes 0..n-1) */
  int32_t fd_order;
} chefsi_grid_t;

/* Kleinman-Bylander projectors (Sec. 2.1, third bullet), all HOST pointers,
 * copied by chefsi_create.  For atom J (0 <= J < n_atoms):
 *   support  S_J = supp_idx[supp_ptr[J] .. supp_ptr[J+1])  linear grid indices,
 *            strictly increasing within an atom;
 *   n_J      = supp_ptr[J+1] - supp_ptr[J];
 *   np_J     = nproj[J] >= 1 projectors;
 *   chi_J    = the next n_J*np_J values of `chi`, column-major n_J x np_J
 *              (projector a of atom J at support point s is chi_J[s + a*n_J]);
 *   gamma_J  = the next np_J values of `gamma` (Ha).
 * n_atoms = 0 means no nonlocal term (the other pointers may then be NULL). */
typedef struct {
  int32_t n_atoms;
  const int64_t* supp_ptr;
  const int32_t* supp_idx;
  const int32_t* nproj;
  const double* chi;
  const double* gamma;
} chefsi_nonlocal_t;

/* Build a handle for one Hamiltonian.  Copies Veff (Nd doubles, HOST) and the
 * projectors to library-owned device memory on the current HIP device (freed
 * by chefsi_destroy); the caller may free its copies on return.  max_ns bounds
 * the ns of later calls.  precision selects the element type of X and the
 * arithmetic of filtering/projection/rotation; the dense stage is always FP64.
 * Returns CHEFSI_ERR_INVALID_ARG on inconsistent input (including a support
 * index outside the grid or not strictly increasing), or with more than 65535
 * projectors in all.  The projector term starts in the stencil pass (records; see
 * chefsi_set_projector_pass) unless the projectors are too many for the block's
 * coefficient row to fit in LDS beside the default tile (in FP64 about 5000 on a grid
 * 120 points wide): the handle then starts on the band pass, and is refused only when a
 * grid point also lies in more than 128 projector supports. */
int chefsi_create(const chefsi_grid_t* grid, const double* veff_host, const chefsi_nonlocal_t* nl,
                  int32_t precision, int32_t max_ns, chefsi_handle_t** out);

/* Replace the handle's local potential (the SCF loop changes Veff between CheFSI calls
 * while grid and projectors stay; Alg. 1 takes H for a given SCF iteration): veff_host
 * holds Nd FP64 values in the grid order of chefsi_create, copied, so the caller may
 * free it on return.  The copies are ordered on `stream`, which is synchronised; work of
 * this handle on other streams must have completed.  chefsi_spectral_bounds and every
 * later call use the new potential.  Errors: ERR_INVALID_ARG (NULL or non-finite
 * values; the handle keeps its old Veff), ERR_HIP. */
int chefsi_update_veff(chefsi_handle_t* h, const double* veff_host, void* stream);

/* Release everything the handle owns.  NULL is ignored. */
void chefsi_destroy(chefsi_handle_t* h);

/* Exact number of workspace bytes every call below needs for block width ns
 * (1 <= ns <= max_ns).  Writes *bytes; used for admission by memory. */
int chefsi_workspace_bytes(const chefsi_handle_t* h, int32_t ns, size_t* bytes);

/* Device bytes the handle itself holds (Veff, projectors and their index
 * tables, copied by chefsi_create); with the orbital block and
 * chefsi_workspace_bytes() this is a request's whole device footprint. */
int chefsi_handle_bytes(const chefsi_handle_t* h, size_t* bytes);

/* Tiling of the fused stencil pass (Sec. 2.1; the paper tiles the stencil for its GPU, this
 * library picks its own tiling at create from the grid shape).  A block of the pass covers
 * whole x rows: row_groups groups of threads, each thread rows_per_thread consecutive rows,
 * so a tile is row_groups * rows_per_thread rows; threads = nx * row_groups (at most 1024
 * for one row per thread, 512 otherwise).  chefsi_set_stencil_tiling(h, 0, 0) restores the
 * library's choice; another pair replaces it (the projector records are rebuilt) and
 * returns CHEFSI_ERR_INVALID_ARG, keeping the current tiling, when it does not fit the
 * grid (rows_per_thread 1..4; the library's own choice uses 1 or 2), or, on the record
 * route, when the tile is too tall for the block's projector coefficients and partial sums
 * in LDS.  Results agree across tilings to rounding (each point
 * sums the same terms; the last bits can differ).  For tuning and tests.
 * chefsi_get_stencil_tiling writes {rows_per_thread, row_groups, tile rows, halo values
 * per thread} to tiling[0..3]. */
int chefsi_set_stencil_tiling(chefsi_handle_t* h, int32_t rows_per_thread, int32_t row_groups);
/* Where the projector term of H X is added (Sec. 2.1, third bullet; results agree to
 * rounding).  in_stencil = 1 (default): points inside at most four projector entries
 * take it inside the stencil pass from per-point records, the others in a separate
 * scatter pass, after a gather of the coefficients over each atom's support.
 * in_stencil = 0 (band pass): the stencil pass runs without records, and one pass over
 * the touched points, region by region (runs of consecutive touched points, each with at
 * most 512 points, 128 projectors and 1920 projector entries), adds every projector term
 * and forms, from the finished values, fixed-order partial sums of the next
 * application's coefficients (the filter carries them from one application to the
 * next).  A grid point inside more than 128 projector supports fits no region: the band
 * pass is then refused with CHEFSI_ERR_INVALID_ARG and the handle stays on the record
 * route; the record route is refused, the handle staying on the band pass, when the
 * current tiling leaves no LDS for its records.  Rebuilds the handle's tables (the band
 * pass holds partial sums for max_ns orbitals on the device); for tuning and tests, not
 * while calls on the handle are in flight. */
int chefsi_set_projector_pass(chefsi_handle_t* h, int32_t in_stencil);

/* Picks the stencil tiling and the projector split by timing them (the planner's
 * tilings of at least r + 1 rows with 1 to 4 rows per thread, each with the projector term
 * in the stencil pass for points inside at most four entries, where the records fit in LDS,
 * and with every term in the band pass): three
 * filter-form H applications per candidate on the first min(ns, 1024) orbitals of the
 * device block X (read only; the workspace block takes the results), on `stream`, which
 * the call synchronises.  Keeps the fastest and, when choice is not NULL, writes
 * {rows per thread, row groups, in_stencil} to choice[0..2] (the band pass is skipped
 * when chefsi_set_projector_pass would refuse it).  Results after tuning agree
 * with the untuned ones to rounding (the same terms summed in another order).  ws as for
 * chefsi_apply_h with this ns.  A one-time set-up call, like a library benchmark mode. */
int chefsi_autotune(chefsi_handle_t* h, const void* X, int32_t ns, void* ws, size_t ws_bytes, void* stream,
                    int32_t* choice);
int chefsi_get_stencil_tiling(const chefsi_handle_t* h, int32_t* tiling);

/* Rigorous filter bounds for the first step (the paper names lam_hi the
 * largest eigenvalue of H and lam_cut the cutoff, Alg. 1, but does not say how
 * they are obtained; these are this library's reading):
 *   lam_hi  = 1/2 sum_d sum_{|p|<=r} |w_p|/h_d^2 + max Veff
 *             + max_i sum_{(J,a) touching i} |gamma_Ja| |chi_Ja(i)| ||chi_Ja||_1 dV   (Gershgorin)
 *   lam_lo  = min Veff (minus the nonlocal bound if some gamma < 0)
 *   lam_cut = lam_lo + 0.1 (lam_hi - lam_lo).
 * Host arithmetic only; any output pointer may be NULL. */
int chefsi_spectral_bounds(const chefsi_handle_t* h, double* lam_lo, double* lam_cut, double* lam_hi);

/* Estimate of lam_Nd, the largest eigenvalue of H (Alg. 1, the top of the filter
 * interval), by `steps` Lanczos steps from the start vector v0 (library reading; the
 * paper does not say how lam_Nd is found):
 *   w = H v_j - beta_{j-1} v_{j-1},  alpha_j = v_j^T w,  w -= alpha_j v_j,
 *   beta_j = ||w||,  v_{j+1} = w / beta_j   (v_1 = v0 / ||v0||, no reorthogonalisation).
 * theta = largest eigenvalue of tridiag(beta, alpha, beta) (a Ritz value, never above
 * lam_Nd); *lam_nd = theta + |beta_k s_k| with s the unit eigenvector of the
 * tridiagonal matrix for theta, i.e. theta plus the Ritz pair's residual norm.
 * v0: device vector of Nd elements in the handle's storage type (FP64 handle: double,
 * mixed handle: float), not modified; products with H and all sums in FP64, orbital
 * vectors stored in the storage type.  ws: caller-owned device memory of
 * chefsi_lanczos_workspace_bytes() bytes.  Synchronises the stream (the coefficients
 * steer the recurrence from the host).  alpha_host/beta_host (optional, `steps`
 * doubles each) receive the coefficients, zeros past an early stop (beta = 0).
 * Errors: ERR_INVALID_ARG (NULL pointers, steps outside 1..1000, zero or non-finite
 * v0), ERR_WORKSPACE, ERR_NONFINITE, ERR_HIP. */
int chefsi_lanczos_workspace_bytes(const chefsi_handle_t* h, size_t* bytes);
int chefsi_lanczos_bound(chefsi_handle_t* h, const void* v0, int32_t steps, void* ws, size_t ws_bytes,
                         void* stream, double* lam_nd, double* theta, double* alpha_host, double* beta_host);

/* Nonlocal (Kleinman-Bylander) part of the Hellmann-Feynman atomic forces, computed the
 * way the paper reuses its filter kernels for forces (Sec. 2: the gradient operator on
 * the orbitals, then the nonlocal projectors on the result):
 *   F_J,d = -2 sum_n g_n sum_a gamma_Ja (dV chi_Ja^T psi_n) (dV chi_Ja^T d psi_n / dx_d),
 * d/dx_d the central FD first derivative of the handle's order 2r (weights
 * c_p = (-1)^(p+1) (r!)^2 / (p (r-p)! (r+p)!), periodic wrap or zero ghosts as the grid).
 * X: ns orbitals psi_n on the device, Nd x ns column-major in the handle's storage type;
 * occ_host: ns occupations g_n; forces_host: n_atoms x 3 doubles (atom-major), written
 * after the stream is synchronised.  FP64 arithmetic throughout.  Forces add over
 * orbitals, so a large block may be passed in column chunks and the results summed.
 * ws: chefsi_forces_workspace_bytes(ns) bytes of device memory (an FP64 Nd x ns
 * gradient block and the projector coefficients).  Errors: ERR_INVALID_ARG,
 * ERR_WORKSPACE, ERR_HIP. */
int chefsi_forces_workspace_bytes(const chefsi_handle_t* h, int32_t ns, size_t* bytes);
int chefsi_nonlocal_forces(chefsi_handle_t* h, const void* X, int32_t ns, const double* occ_host, void* ws,
                           size_t ws_bytes, void* stream, double* forces_host);

/* Electronic kinetic-energy component of the stress from the same FD gradient of the
 * orbitals (Sec. 2 names this reuse of the gradient for the stresses):
 *   sigma_ab = -(1 / Omega) sum_n g_n dV sum_i (d psi_n/dx_a)(i) (d psi_n/dx_b)(i),
 * Omega = Nd dV, in Ha / bohr^3.  X, occ_host, ws as chefsi_nonlocal_forces (the same
 * workspace size); stress_host: 9 doubles, row-major 3 x 3 (symmetric), written after the
 * stream is synchronised.  Fixed-order sums (bitwise reproducible).  Errors as above. */
int chefsi_kinetic_stress(chefsi_handle_t* h, const void* X, int32_t ns, const double* occ_host, void* ws,
                          size_t ws_bytes, void* stream, double* stress_host);

/* Nonlocal (Kleinman-Bylander) component of the stress, the other quantity Sec. 2 computes
 * with the gradient of the orbitals followed by the nonlocal projectors.  Under a
 * homogeneous strain the projectors are sampled at the strained displacement from their
 * atom; the strain derivative of E_nl = sum_n g_n sum_{J,a} gamma_Ja (dV chi_Ja^T psi_n)^2,
 * integrated by parts over each support, is
 *   sigma_ab = -(1 / Omega) [delta_ab E_nl + 2 sum_n g_n sum_{J,a} gamma_Ja alpha beta_ab],
 *   alpha = dV chi_Ja^T psi_n,  beta_ab = dV sum_i chi_Ja(i) d_b(i) (d psi_n / dx_a)(i),
 * d/dx_a the handle's central FD first derivative, Omega = Nd dV (Ha / bohr^3).
 * disp_host: HOST, 3 doubles per support point in the order of chefsi_nonlocal_t.supp_idx
 * (atom by atom), the displacement d = r_i - R_J of the point from its atom (the minimum
 * image the projector values were evaluated at); may be NULL when the handle has no
 * projectors.  X, occ_host, ws (chefsi_forces_workspace_bytes) as chefsi_nonlocal_forces;
 * stress_host: 9 doubles, row-major (a, b), written after the stream is synchronised.  Not
 * symmetric in general: it is when the projector set of every atom is closed under
 * rotations (e.g. equal energies within an l shell).  FP64 arithmetic; fixed-order sums.
 * Errors: ERR_INVALID_ARG (NULL pointers, non-finite occupations or displacements),
 * ERR_WORKSPACE, ERR_HIP. */
int chefsi_nonlocal_stress(chefsi_handle_t* h, const void* X, int32_t ns, const double* occ_host,
                           const double* disp_host, void* ws, size_t ws_bytes, void* stream, double* stress_host);

/* Y = H X for an Nd x ns block (Sec. 2.1: stencil + Veff + nonlocal).  X and Y
 * are distinct device blocks of the handle's element type. */
int chefsi_apply_h(chefsi_handle_t* h, const void* X, void* Y, int32_t ns,
                   void* ws, size_t ws_bytes, void* stream);

/* Size of the library's static device scratch (64 MiB per GPU, held from the first
 * chefsi_create on that GPU until the process ends). */
#define CHEFSI_STATIC_SCRATCH_BYTES (64u << 20)

/* For callers that cannot allocate device memory (code under HIP graph capture,
 * serving loops that must not call hipMalloc, harnesses that forbid it): Y = H X
 * exactly as chefsi_apply_h computes it (same kernels, same bits), with the
 * projector coefficients alpha (np_tot x ns values of the handle's element type) in
 * the library's static per-GPU scratch instead of a caller workspace.  The call
 * allocates nothing (no hipMalloc/hipFree, no allocating library routine, no event
 * creation) and only enqueues kernels on `stream`.  X and Y are distinct caller-owned
 * device blocks (Nd x ns, ld Nd, the handle's element type).
 * Limit: np_tot * ns * sizeof(element) <= CHEFSI_STATIC_SCRATCH_BYTES (query it with
 * chefsi_static_scratch_bytes); larger requests return CHEFSI_ERR_WORKSPACE before any
 * launch (call on fewer orbitals at a time).  Every call on one GPU shares that GPU's
 * scratch: calls that overlap on one GPU (other streams, other threads, other
 * handles) race and must be serialised by the caller.  The scratch is fully written
 * before it is read in each call; nothing carries over from the previous call. */
int chefsi_static_scratch_bytes(const chefsi_handle_t* h, int32_t ns, size_t* bytes);
int chefsi_apply_h_static(chefsi_handle_t* h, const void* X, void* Y, int32_t ns, void* stream);

/* X <- scaled Chebyshev filter of degree m >= 1 applied to X, in place
 * (Alg. 1, Filtering).  Requires lam_lo < lam_cut < lam_hi. */
int chefsi_filter(chefsi_handle_t* h, void* X, int32_t ns, int32_t degree,
                  double lam_lo, double lam_cut, double lam_hi,
                  void* ws, size_t ws_bytes, void* stream);

/* Projection (Alg. 1; Sec. 2.2): Hs = X^T (H X) and Ms = X^T X for the
 * filtered block X, written as full symmetric ns x ns column-major FP64
 * matrices to the device arrays Hs and Ms (leading dimension ns). */
int chefsi_project(chefsi_handle_t* h, const void* X, int32_t ns, double* Hs, double* Ms,
                   void* ws, size_t ws_bytes, void* stream);

/* Subspace diagonalization (Alg. 1; Sec. 2.3): solve Hs Z = Ms Z D in FP64 on
 * the device.  Hs and Ms (device, ns x ns, ld ns, symmetric; upper triangles
 * read) are overwritten: Hs by Z (Z^T Ms Z = I, columns ordered by ascending
 * D), Ms by the Cholesky factor of S Ms S, where S = diag(Ms_ii^-1/2) scales the
 * pencil before the factorization (it leaves D unchanged and keeps the
 * Cholesky usable when the filtered columns differ widely in norm).  D
 * (device, ns doubles) gets the eigenvalues in ascending order.
 * CHEFSI_ERR_NOT_POSDEF if Ms is not positive definite. */
int chefsi_eigh(chefsi_handle_t* h, double* Hs, double* Ms, double* D, int32_t ns,
                void* ws, size_t ws_bytes, void* stream);

/* Rotation (Alg. 1; Sec. 2.4): X <- X Z for a device ns x ns FP64 matrix Z
 * (column-major, ld ns), in place. */
int chefsi_rotate(chefsi_handle_t* h, void* X, const double* Z, int32_t ns,
                  void* ws, size_t ws_bytes, void* stream);

/* One whole CheFSI step (Alg. 1): filter, project, diagonalize, rotate.  X is
 * updated in place to the rotated block X~ Z~ (orthonormal columns, ordered by
 * ascending Ritz value); ritz_host (HOST, ns doubles) receives D~.  Returns
 * CHEFSI_ERR_NONFINITE if a Ritz value is not finite. */
int chefsi_step(chefsi_handle_t* h, void* X, int32_t ns, int32_t degree,
                double lam_lo, double lam_cut, double lam_hi,
                void* ws, size_t ws_bytes, void* stream, double* ritz_host);

/* n_iter >= 1 CheFSI steps from X with the bounds update used between SCF
 * iterations by this library (a reading; the paper fixes none):
 * lam_lo <- D_1 and lam_cut <- D_ns after every step, lam_hi fixed.
 * ritz_host receives the last step's D~.  The final bounds are written to
 * *lam_lo_out / *lam_cut_out when those are not NULL. */
int chefsi_solve(chefsi_handle_t* h, void* X, int32_t ns, int32_t degree, int32_t n_iter,
                 double lam_lo, double lam_cut, double lam_hi,
                 void* ws, size_t ws_bytes, void* stream, double* ritz_host,
                 double* lam_lo_out, double* lam_cut_out);

/* Final FP64 Rayleigh-Ritz pass (the mixed-precision path ends with it; the
 * paper's own steps are FP64 throughout, Sec. 2).  With degree > 0 the block is
 * first filtered (Alg. 1, Filtering; storage precision, bounds as for
 * chefsi_filter), which also damps what the split-bf16 rotation of the previous
 * step left outside the wanted subspace; degree == 0 skips the filter and
 * ignores the bounds.  Then Hs = X^T (H X) and Ms = X^T X are formed with FP64
 * arithmetic from the stored block, the FP64 subspace problem is solved, X is
 * rotated in FP64 (stored back once rounded to the handle's element type) and
 * ritz_host (HOST, ns doubles) receives the FP64 Ritz values.  On a
 * CHEFSI_FP64 handle with degree > 0 this equals chefsi_step. */
int chefsi_refine_fp64(chefsi_handle_t* h, void* X, int32_t ns, int32_t degree,
                       double lam_lo, double lam_cut, double lam_hi,
                       void* ws, size_t ws_bytes, void* stream, double* ritz_host);

/* Per-kernel timing with HIP events recorded on the call's stream around every
 * launch of the named kernel (off by default; enabling it adds event records
 * but changes no result).  kernel ids: 0 hx_apply, 1 nl_project, 2 gram,
 * 3 gram_reduce, 4 rotate, 5 dense eigensolve (whole FP64 stage), 6 copy,
 * 7 mixed steps redone in FP64 (count only, kept whether or not timing is on:
 * a mixed step whose scaled overlap matrix has a Cholesky pivot below 1e-4, or
 * no Cholesky, forms its projection and rotation with FP64 arithmetic instead).
 * chefsi_profile_read synchronizes on the recorded events and returns the
 * summed milliseconds and launch count since the last reset. */
int chefsi_profile_enable(chefsi_handle_t* h, int32_t on);
int chefsi_profile_reset(chefsi_handle_t* h);
int chefsi_profile_read(chefsi_handle_t* h, int32_t kernel_id, double* total_ms, int64_t* launches);

/* Status of the last failing call on this handle: for NOT_POSDEF the
 * rocSOLVER info value (order of the failing leading minor + ns), else 0. */
int chefsi_last_info(const chefsi_handle_t* h);

/* Static description of a status code, and the last error message recorded on
 * a handle (never NULL; empty if none). */
const char* chefsi_strerror(int status);
const char* chefsi_last_error(const chefsi_handle_t* h);

/* Library version as MAJOR*10000 + MINOR*100 + PATCH. */
int chefsi_version(void);

/* ---- CheFSI at a Bloch wavevector (complex FP64) ----------------------------
 * Sec. 2 of the paper: Gamma-point and isolated systems run in real arithmetic,
 * every other Brillouin-zone sample in complex double precision; H of Alg. 1 is
 * the Hamiltonian of one Bloch wavevector k (bohr^-1).  Orbitals are Bloch
 * periodic, psi(r + L_d e_d) = exp(i k_d L_d) psi(r), L_d = n_d h_d, in every
 * periodic direction (k_d is ignored in Dirichlet ones):
 *   - the FD ghosts of Sec. 2.1 across a periodic face carry exp(+-i k_d L_d);
 *   - every projector is its Bloch sum: the value of support point s of atom J
 *     becomes chi_J(s) exp(i k.(m_s L)), where m_s (supp_img[3 s .. 3 s + 2],
 *     HOST int32, one triple per support point in supp_idx order) is the lattice
 *     image the point belongs to: point = R_J + m_s L + the displacement chi_J
 *     was evaluated at (the truncation radius must be below half the cell so a
 *     point sees one image);
 *   - V_nl psi = sum_J chi~_J Gamma_J (chi~_J^H psi[S_J]) dV.
 * Blocks are DEVICE, complex FP64 with interleaved real and imaginary parts
 * (re, im), Nd x ns column major (ld = Nd): a torch.complex128 tensor of shape
 * (ns, Nd).  A step is Alg. 1 with conjugate transposes: Hs = X~^H H X~,
 * Ms = X~^H X~, Hs Z = Ms Z D (Hermitian definite, ascending D), X = X~ Z.
 * The projector term is added by a band pass like the real handle's (see
 * chefsi_set_projector_pass), so a grid point may lie in at most 128 projector supports
 * (CHEFSI_ERR_INVALID_ARG at create otherwise).
 * The handle holds its own copies of all host inputs (freed by
 * chefsi_kpoint_destroy); calls are ordered on their stream; Nd < 2^31 and
 * max_ns <= min(Nd, 65535) (CHEFSI_ERR_INVALID_ARG otherwise); a block may hold
 * 2^31 elements or more (the rotation runs in row panels below that size).
 * Errors as for the real handle (INVALID_ARG, WORKSPACE, NOT_POSDEF, EIG,
 * NONFINITE, SOLVER, HIP, OOM); after an error the handle stays usable and X
 * is unspecified. */
typedef struct chefsi_kpoint chefsi_kpoint_t;

int chefsi_kpoint_create(const chefsi_grid_t* grid, const double* veff_host, const chefsi_nonlocal_t* nl,
                         const int32_t* supp_img, const double* kvec, int32_t max_ns, chefsi_kpoint_t** out);
void chefsi_kpoint_destroy(chefsi_kpoint_t* h);
const char* chefsi_kpoint_last_error(const chefsi_kpoint_t* h);

/* Exact device workspace (bytes, 256-byte aligned base required) of the calls below. */
int chefsi_kpoint_workspace_bytes(chefsi_kpoint_t* h, int32_t ns, size_t* bytes);

/* Y = H_k X (X and Y distinct device blocks of ns orbitals). */
int chefsi_kpoint_apply_h(chefsi_kpoint_t* h, const void* X, void* Y, int32_t ns, void* ws, size_t ws_bytes,
                          void* stream);

/* One complex CheFSI step (Alg. 1): the scaled Chebyshev filter of degree >= 1
 * with bounds lam_lo <= lam_cut < lam_hi, projection, Hermitian-definite
 * eigensolve, rotation.  X is updated in place; ritz_host (HOST, ns doubles)
 * receives D ascending. */
int chefsi_kpoint_step(chefsi_kpoint_t* h, void* X, int32_t ns, int32_t degree, double lam_lo, double lam_cut,
                       double lam_hi, void* ws, size_t ws_bytes, void* stream, double* ritz_host);

/* Per-kernel timing of a k-point handle, as chefsi_profile_* for the real handle (HIP
 * events on the call's stream, off by default, no effect on results).  kernel ids:
 * 0 zhx (Bloch-phased stencil pass), 1 band passes (projector scatter and coefficient
 * gather, with their reductions), 2 projection (zgemm batches and the partial sums),
 * 3 dense stage (zpotrf, ztrsm, zheevd), 4 rotation (zgemm row panels and the copy
 * back).  chefsi_kpoint_profile_read synchronizes on the recorded events and returns
 * the summed milliseconds and launch count since the last reset; ids outside 0..4 are
 * CHEFSI_ERR_INVALID_ARG. */
int chefsi_kpoint_profile_enable(chefsi_kpoint_t* h, int32_t on);
int chefsi_kpoint_profile_reset(chefsi_kpoint_t* h);
int chefsi_kpoint_profile_read(chefsi_kpoint_t* h, int32_t kernel_id, double* total_ms, int64_t* launches);

#ifdef __cplusplus
}
#endif

#endif /* CHEFSI_H */
