/*
 * rsdft.h - C ABI of the MI355X (gfx950) real-space Kohn-Sham hot path.
 *
 * Implements the data-parallel core of Andrade & Aspuru-Guzik, "Real-space
 * density functional theory on graphical processing units" (arXiv 1306.2953):
 * applying the Kohn-Sham Hamiltonian to blocks of states on an irregular grid
 * (Sec. 5), and the orthogonalisation and subspace diagonalisation that the
 * RMM-DIIS eigensolver wraps around it (Secs. 3 and 6).
 *
 * Conventions shared by every call
 * --------------------------------
 *  - Every function returns an rs_status; 0 (RS_OK) is success.  On failure
 *    rs_last_error() gives a message (thread-local, valid until the next
 *    call on the same thread).  No C++ exception crosses this boundary.
 *  - Field arrays are caller-owned DEVICE memory on the current HIP device,
 *    contiguous, 16-byte aligned, in the "block of states" layout of Sec. 4
 *    (Fig. "memory_layout" (b)): psi[blk][point][B], the B states of a block
 *    stored contiguously for each grid point, blocks one after another.
 *    B is a power of two, 1 <= B <= 64 (Sec. 4: block size is chosen at run
 *    time and restricted to small powers of two).  Points are the grid's
 *    inner points in index-map order (rs_grid_export); values outside the
 *    domain are zero (finite systems) or periodic images (periodic box) and
 *    are never stored.
 *  - dtype selects the storage type of fields: RS_F64 (double) or RS_F32
 *    (float).  Small matrices (overlap, subspace Hamiltonian, Cholesky
 *    factor, eigenvectors, eigenvalues) are always double.  rs_hpsi_block,
 *    rs_project_nl, rs_apply_nl and rs_overlap also take complex states
 *    (eq. (1b) conjugates them): RS_C128 (double re, im) and RS_C64 (float
 *    re, im), the two parts interleaved, so a block of B complex states is
 *    laid out as a block of 2B real columns (re of state 0, im of state 0,
 *    re of state 1, ...); B <= 32.
 *  - Host arrays passed to *_create calls are copied; handles own their
 *    device tables and scratch, sized at creation, so the field calls never
 *    allocate device memory.
 *  - `stream` is a hipStream_t (0 = the null stream).  Field calls only
 *    enqueue work on it and return without waiting, unless stated.
 *  - The grid inner product is <f|g> = h^3 sum_p f(p) g(p) (the integral of
 *    eq. (6) and eqs. (7), (9) replaced by a grid sum).
 */
#ifndef RSDFT_H
#define RSDFT_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int rs_status;
#define RS_OK          0
#define RS_EINVAL      1  /* bad argument (null, size, alignment, B, dtype) */
#define RS_ENOTPOSDEF  2  /* overlap matrix not positive definite          */
#define RS_ENONFINITE  3  /* a non-finite value was produced or found      */
#define RS_EHIP        4  /* HIP runtime failure                           */
#define RS_ENOMEM      5  /* device or host allocation failure             */
#define RS_ENOTSUP     6  /* valid but unsupported combination             */
#define RS_ENOTCONV    7  /* an iteration did not reach its tolerance      */

#define RS_F64 0
#define RS_F32 1
#define RS_C128 2   /* complex, double parts */
#define RS_C64 3    /* complex, float parts  */

/* Contraction precision of the point-summed products (overlap, subspace
 * matrix, rotations).  RS_PREC_NATIVE: the storage type, with FP64
 * accumulation of the split-K partial sums.  RS_PREC_BF16X3: FP32 fields
 * split as a = a_hi + a_lo (each bfloat16, round to nearest even); products
 * on matrix cores with FP32 accumulation.  Overlaps: a_hi b_hi + a_hi b_lo +
 * a_lo b_hi + a_lo b_lo (the last keeps norms unbiased) summed in FP32 over
 * at most 32 points per matrix-core step, the steps accumulated in FP64.
 * Rotations: field and FP64 matrix
 * are both split in three bfloat16 terms and the six products a_i x_j with
 * i + j <= 2 are summed in FP32, which keeps the rotated field at FP32
 * accuracy. */
#define RS_PREC_NATIVE 0
#define RS_PREC_BF16X3 1

const char *rs_last_error(void);
int rs_version(void);

/* ------------------------------------------------------------------ grid
 * Sec. 2 / Sec. 5.1: a uniform grid of spacing h restricted to a shape, with
 * points enumerated by small parallelepipedic sub-grids ("bricks",
 * Fig. "locality" (b)).
 *
 * kind  RS_GRID_BOX:      n^3 points, cell-centred (x_i = (i - (n-1)/2) h),
 *                         zero outside (finite system).
 *       RS_GRID_PERIODIC: n^3 points, x_i = i h, periodic with L = n h;
 *                         n must be a multiple of each brick edge.
 *       RS_GRID_SPHERE:   points (i, j, k) h with i^2 + j^2 + k^2 <= Q, where
 *                         Q = q^2 if R/h equals an integer q to 1e-9 relative
 *                         and floor((R/h)^2) otherwise; zero outside.
 *       RS_GRID_UNION:    the molecular grid of Sec. 2 (Fig. "struct"): the
 *                         points (i, j, k) h inside at least one sphere of
 *                         radius R around the natoms centres (X, Y, Z),
 *                         ((i h - X)^2 + (j h - Y)^2) + (k h - Z)^2 <= R^2 in
 *                         FP64 rounded as written; zero outside.  The
 *                         lattice spans floor((min X - R)/h) ..
 *                         ceil((max X + R)/h) per axis (plus 4 each side).
 * brick: sub-grid edge lengths (>= 1).  The kernels of this library require
 *        the default 4 x 4 x 4; other shapes only change the index map.
 * Ordering: bricks x fastest, then y, then z over the brick lattice (which
 * starts 4 points before the domain on each side for finite systems);
 * inside a brick x is fastest.  Inner points come first; "boundary" points
 * (outside, within 4 steps of an inner point along one axis) are listed
 * separately by rs_grid_export and are implicit zeros in every kernel.
 */
#define RS_GRID_BOX      0
#define RS_GRID_PERIODIC 1
#define RS_GRID_SPHERE   2
#define RS_GRID_UNION    3

typedef struct rs_grid rs_grid;

typedef struct {
    int32_t kind;
    double  h;         /* spacing (bohr), > 0                      */
    int32_t n;         /* edge in points (box, periodic)           */
    double  radius;    /* sphere radius (bohr)                     */
    int32_t brick[3];  /* sub-grid edges; {0,0,0} selects 4,4,4    */
    int32_t flags;     /* RS_GRID_HOST_ONLY: build the index map on  */
                       /* the host only (no device tables; field     */
                       /* calls on such a grid return RS_EINVAL)     */
    int32_t natoms;    /* union: number of sphere centres (>= 1)   */
    const double *centres;  /* union: HOST [natoms][3] bohr, copied */
} rs_grid_desc;

#define RS_GRID_HOST_ONLY 1

/* Builds the index map on the host and uploads the brick tables to the
 * current device (unless RS_GRID_HOST_ONLY).  Errors: RS_EINVAL for a bad
 * descriptor, RS_EHIP / RS_ENOMEM from the upload. */
rs_status rs_grid_create(const rs_grid_desc *desc, rs_grid **out);
void rs_grid_destroy(rs_grid *g);

/* Sizes: inner points, boundary points, numbered bricks (those holding an
 * inner point), brick-lattice counts nb[3] (x, y, z) and the integer
 * coordinate lo[3] of the lattice origin.  Any pointer may be NULL. */
rs_status rs_grid_info(const rs_grid *g, int64_t *np, int64_t *nbnd,
                       int64_t *nbricks, int32_t nb[3], int32_t lo[3]);

/* Host copies of the index map: integer coordinates of inner [np][3] and
 * boundary [nbnd][3] points (x, y, z), the brick map [nb2][nb1][nb0] (brick
 * number or -1), and physical coordinates of inner points [np][3] in bohr.
 * Any pointer may be NULL. */
rs_status rs_grid_export(const rs_grid *g, int32_t *inner, int32_t *boundary,
                         int32_t *brick_map, double *xyz);

/* ------------------------------------------------------- non-local part
 * Eq. (6), Sec. 5.3, with a diagonal coupling: V_nl = sum_A sum_i
 * |gamma_A,i> D_A,i <gamma_A,i|, i running over the (lmax+1)^2 pairs (l, m),
 * l = 0..lmax <= 3, m = -l..l:
 *   gamma_lm(r) = N_l r^l Y_lm(r/|r|) exp(-r^2 / 2 sigma^2),
 * Y_lm the real spherical harmonics (unit-normalised on the sphere) and
 * N_l = (Gamma(l + 3/2) sigma^(2l+3) / 2)^(-1/2), so that each gamma has
 * unit continuum norm; nonzero for |r_p - R_A|^2 <= rc^2 (minimum image on
 * periodic grids).  Projector order within an atom: l ascending; l = 1:
 * x, y, z; l = 2: xy, yz, 3z^2 - r^2, xz, x^2 - y^2; l = 3: y(3x^2 - y^2),
 * xyz, y(5z^2 - r^2), z(5z^2 - 3r^2), x(5z^2 - r^2), z(x^2 - y^2),
 * x(x^2 - 3y^2).  lmax = 1 is the s, p_x, p_y, p_z set
 * (N_s exp(-r^2/2 sigma^2), N_p r_a exp(-r^2/2 sigma^2)).  Atoms are split
 * into colour groups with disjoint spheres (greedy, atom order; Fig.
 * "colors").  The projectors are real, so a complex state's projections
 * are those of its real and imaginary parts.
 *
 * pos [nat][3] (bohr) and D [nat][(lmax+1)^2] (Ha) are host arrays.
 * max_states is the largest number of real state columns later passed to
 * the field calls (nblk*B, or 2*nblk*B for complex states; sizes scratch).
 * On a host-only grid the set is built on the host only (export works,
 * field calls return RS_EINVAL).  Errors: RS_EINVAL (null, nat < 0, rc or
 * sigma <= 0, lmax outside 0..3, max_states outside 1..4096). */
typedef struct rs_nl rs_nl;
rs_status rs_nl_create(const rs_grid *g, int32_t nat, const double *pos,
                       const double *D, double rc, double sigma, int32_t lmax,
                       int32_t max_states, rs_nl **out);
void rs_nl_destroy(rs_nl *nl);
/* Total sphere entries, number of colour groups and projectors per atom
 * ((lmax+1)^2); any pointer may be NULL. */
rs_status rs_nl_info(const rs_nl *nl, int64_t *nnz, int32_t *ncolours, int32_t *nproj);
/* Host copies: sph_ptr [nat+1], sph_idx [nnz] (inner-point indices, ascending
 * per atom), gamma [nnz][nproj], colour [nat].  Any pointer may be NULL. */
rs_status rs_nl_export(const rs_nl *nl, int64_t *sph_ptr, int64_t *sph_idx,
                       double *gamma, int32_t *colour);

/* ------------------------------------------------------------- H psi
 * Sec. 5: hpsi = (T + V + V_nl) psi for nblk blocks of B states.
 *   T: -1/(2h^2) sum_axes sum_{m=1..4} c_m [(psi(p+m e) - psi(p)) +
 *      (psi(p-m e) - psi(p))], c = (8/5, -1/5, 8/315, -1/560), the 25-point
 *      star of Sec. 5.1 (equal to the c_0 form since c_0 = -2 sum c_m);
 *   V: vloc [np] (dtype), Sec. 5.2;
 *   V_nl: eq. (6) when nl != NULL (projections, then the point-centric sum
 *      over the atoms whose sphere holds the point; no atomics).
 * psi [nblk][np][B] and hpsi [nblk][np][B] must not overlap.  Asynchronous.
 * Complex dtypes: H is real, so each complex state is applied as its real
 * and imaginary columns (B <= 32).
 * Errors: RS_EINVAL (B, dtype, pointers, nblk*B real columns > max_states
 * of nl), RS_ENOTSUP (brick other than 4x4x4). */
rs_status rs_hpsi_block(const rs_grid *g, const rs_nl *nl, const void *vloc,
                        const void *psi, void *hpsi, int32_t nblk, int32_t B,
                        int32_t dtype, void *stream);

/* First part of eq. (6): proj[blk][A][i][s] = h^3 sum_{p in sphere A}
 * gamma_A,i(p) psi[blk][p][s] (D not applied), i < nproj, FP64
 * accumulation, stored in dtype (complex: proj[blk][A][i][s] complex, the
 * real layout with 2B columns).  Asynchronous. */
rs_status rs_project_nl(const rs_grid *g, const rs_nl *nl, const void *psi,
                        void *proj, int32_t nblk, int32_t B, int32_t dtype,
                        void *stream);

/* Second part of eq. (6): hpsi[blk][p][s] += sum_{A : p in sphere A}
 * sum_i gamma_A,i(p) D_A,i proj[blk][A][i][s], i < nproj (complex states as
 * in rs_project_nl).  Asynchronous. */
rs_status rs_apply_nl(const rs_grid *g, const rs_nl *nl, const void *proj,
                      void *hpsi, int32_t nblk, int32_t B, int32_t dtype,
                      void *stream);

/* -------------------------------------------- orthogonalisation, Sec. 6
 * A context holds the workspaces of the point-summed contractions and the
 * small FP64 matrices for up to max_states (<= 256) states of one grid.
 * Field calls on one context must not overlap in time (shared scratch). */
typedef struct rs_ctx rs_ctx;
rs_status rs_ctx_create(const rs_grid *g, int32_t max_states, rs_ctx **out);
void rs_ctx_destroy(rs_ctx *c);

/* Eq. (7) generalised: S[j][k] = h^3 sum_p X[p][j] Y[p][k] for N = nblk*B
 * states stored in the block layout; S is DEVICE double [N][N].  When x == y
 * only the upper 16x16 blocks are formed (symmetric rank-k product) and
 * mirrored.  The points are split in chunks (a few hundred to a few
 * thousand points each, set by the grid and the shape); the chunks' partial
 * sums are added in FP64 in a fixed order (bitwise repeatable for a given
 * grid and shape).  prec must be RS_PREC_NATIVE for RS_F64
 * and RS_PREC_BF16X3 for RS_F32 (else RS_ENOTSUP).  Complex states (RS_C128
 * with RS_PREC_NATIVE, RS_C64 with RS_PREC_BF16X3): S is DEVICE complex
 * double [N][N] (re, im interleaved), S[j][k] = h^3 sum_p conj(X[p][j])
 * Y[p][k], formed from the real products of the 2N real columns; needs
 * 2N <= max_states.  Asynchronous. */
rs_status rs_overlap(rs_ctx *c, const void *x, const void *y, double *S, int32_t nblk,
                     int32_t B, int32_t dtype, int32_t prec, void *stream);

/* rs_overlap for callers that cannot allocate device memory (code under HIP
 * graph capture, serving loops, harnesses that forbid hipMalloc): the same
 * product S = h^3 X^T Y (DEVICE double [N][N]) with no context.  Its chunk
 * partial sums, group sums and block lists live in a fixed 64 MiB device
 * array that the library holds on each GPU it runs on until the process
 * ends; the call performs no allocation of any kind.  Limits: N = nblk*B in
 * [1, 256] (else RS_EINVAL); the chunks grow when the array holds fewer
 * partial sums than rs_overlap would use (for 256 states, grids above about
 * 450k points), which changes only the rounding.  Every call on a GPU uses
 * that GPU's one
 * array, whose contents the last call leaves behind (nothing in it needs to
 * start at zero): calls that overlap in time on one GPU (any streams, any
 * threads) race and give wrong results.  The array's device address is
 * looked up once per device, on the first call made with it current.
 * Real dtypes only (RS_F64, RS_F32; complex dtypes return RS_EINVAL);
 * errors otherwise as rs_overlap.  Asynchronous. */
rs_status rs_overlap_noalloc(const rs_grid *g, const void *x, const void *y, double *S,
                             int32_t nblk, int32_t B, int32_t dtype, int32_t prec,
                             void *stream);

/* psi <- psi X in place (eqs. (8) and (10): new state c = sum_n X[n][c] old
 * state n); X is DEVICE double [N][N].  Asynchronous. */
rs_status rs_rotate(rs_ctx *c, void *psi, const double *X, int32_t nblk, int32_t B,
                    int32_t dtype, int32_t prec, void *stream);

/* S = U^T U (Sec. 6), U upper triangular with positive diagonal, all DEVICE
 * double [N][N]; *info (DEVICE int) = 0 or the 1-based column whose pivot is
 * not positive (LAPACK potrf convention).  Asynchronous. */
rs_status rs_cholesky(rs_ctx *c, const double *S, double *U, int32_t N, int32_t *info,
                      void *stream);

/* Symmetric eigenproblem A V = V diag(evals) by cyclic Jacobi in the
 * parallel round-robin order (FP64, DEVICE arrays; A [N][N] must be exactly
 * symmetric and is destroyed).  Eigenvalues ascending; column j of V is
 * eigenvector j with its largest-magnitude component positive.
 * Asynchronous. */
rs_status rs_eigh(rs_ctx *c, double *A, double *V, double *evals, int32_t N, void *stream);

/* Sec. 6, eqs. (7)-(8): S = <psi|psi>, S = U^T U, psi <- psi U^-1 (so the new
 * states are orthonormal and state j spans the first j old states).  S_out
 * (DEVICE double [N][N]) may be NULL.  Synchronises the stream to read the
 * Cholesky status: on a non-positive pivot returns RS_ENOTPOSDEF with *info
 * (HOST int, may be NULL) the 1-based column, and leaves psi unchanged. */
rs_status rs_orthonormalize_block(rs_ctx *c, void *psi, int32_t nblk, int32_t B,
                                  int32_t dtype, int32_t prec, double *S_out, int32_t *info,
                                  void *stream);

/* Sec. 6, eqs. (9)-(10): h = (M + M^T)/2, M = <psi|hpsi>; h = V diag(eig) V^T;
 * psi <- psi V and hpsi <- hpsi V in place; eig is DEVICE double [N],
 * ascending.  Asynchronous. */
rs_status rs_subspace_diag(rs_ctx *c, void *psi, void *hpsi, double *eig, int32_t nblk,
                           int32_t B, int32_t dtype, int32_t prec, void *stream);

/* --------------------------------------------- Hartree potential, Sec. 7
 * Eq. (5): V_H solves nabla^2 V = -4 pi n; for a finite system V(r) =
 * int n(r') / |r - r'| d^3r'.  The density on the grid's inner points is
 * placed in an N^3 box (zeros elsewhere), transformed by a 3-D FFT,
 * multiplied by the Coulomb interaction cut off at R_c,
 *     v(k) = 4 pi / k^2 (1 - cos(k R_c)),  v(0) = 2 pi R_c^2,
 * transformed back and read out at the inner points.  R_c = twice the
 * largest distance of an inner point from the centre of their bounding box
 * (so it bounds every pair distance); N = the smallest power of two with
 * N > (extent - 1) + R_c / h on every axis (the box then keeps every
 * periodic image of the density more than R_c from the domain), at least
 * 16 and at most 512 (RS_ENOTSUP beyond).  FP64 throughout.  Finite grids
 * only (RS_EINVAL for periodic ones).  The handle owns the box (16 N^3
 * bytes) and the point table; it holds a pointer to the grid, which must
 * outlive it. */
typedef struct rs_poisson rs_poisson;
rs_status rs_poisson_create(const rs_grid *g, rs_poisson **out);
void rs_poisson_destroy(rs_poisson *p);
/* The box edge N and R_c (bohr) chosen at creation (HOST outputs, may be
 * NULL). */
rs_status rs_poisson_info(const rs_poisson *p, int32_t *nbox, double *rc);
/* vh[p] = V_H at inner point p for the density rho[p]; rho, vh DEVICE
 * double [np], distinct.  Calls on one handle must not overlap in time (one
 * box).  Asynchronous. */
rs_status rs_poisson_solve(rs_poisson *p, const double *rho, double *vh, void *stream);

/* ------------------------------------------------- eigensolver, Sec. 3
 * RMM-DIIS with the filter preconditioner and the block stopping rule of
 * Sec. 9.  One rs_eigensolve_step:
 *   1. H psi for all states; Rayleigh-Ritz (eqs. (9)-(10)); eig = its
 *      eigenvalues (ascending).
 *   2. Per state: eps0 = <psi|H psi>/<psi|psi>, R0 = H psi - eps0 psi,
 *      resnorm = ||R0||.  A block whose states all have resnorm < tol is
 *      frozen for the rest of the step (when block_stop).
 *   3. d = K R0 with K r = alpha r + (1 - alpha)/6 (sum of the six nearest
 *      neighbours); lambda minimises the Rayleigh quotient of psi + lambda d;
 *      psi_1 = psi + lambda d.
 *   4. For j = 1 .. m-1: the residuals R_i = H psi_i - eps_i psi_i of the
 *      iterates so far are combined with coefficients c minimising
 *      ||sum c R|| / ||sum c psi|| (lowest generalised eigenvector, written in
 *      the basis {psi_L, psi_i - psi_L}, c_0 = 1); psi_{j+1} = sum c psi +
 *      lambda K (sum c R), H psi_{j+1} updated linearly.
 *   5. psi <- newest iterate, then orthonormalised (Cholesky, eq. (8)).
 * Applications of H per step: 1 + m.  FP32 fields use the split-BF16
 * contractions of RS_PREC_BF16X3; every inner product is accumulated in
 * FP64 and the small per-state problems are solved in FP64. */
typedef struct rs_solver rs_solver;
typedef struct {
    int32_t m;           /* iterates built per step (H d applications), 1..3 */
    double  alpha;       /* filter centre weight (0.52)                      */
    double  tol;         /* residual threshold of the block stopping rule    */
    int32_t block_stop;  /* nonzero: freeze blocks whose states are all < tol */
    int32_t record;      /* nonzero: keep R0 and sigma of each step for
                            rs_eigensolve_residuals (training data)          */
    int32_t rr_sweeps;   /* Jacobi sweep cap of the step's Rayleigh-Ritz
                            problem, 1..30; 0 (default): 30, i.e. sweeps run
                            until the off-diagonal norm is below 1e-15 of the
                            matrix norm (converged to FP64 accuracy)          */
} rs_solver_opts;

/* nstates (<= 256) states of dtype in nblk = ceil(nstates / B) blocks on
 * grid g with local potential vloc (DEVICE [np] of dtype; must stay valid
 * for the solver's lifetime) and optional projectors nl (max_states >=
 * nblk * B).  When B does not divide nstates the last block is padded with
 * zero states: they stay zero, get identity pivots in the orthonormalisation
 * and are left out of the Rayleigh-Ritz problem, the stopping rule and the
 * outputs.  opts NULL: m = 3, alpha = 0.52,
 * tol = 1e-6, block_stop = 1, record = 0, rr_sweeps = 0.  Allocates all workspaces (about 2(m+1)+3
 * field arrays of np * nstates elements). */
rs_status rs_eigensolve_create(const rs_grid *g, const rs_nl *nl, const void *vloc,
                               int32_t nstates, int32_t B, int32_t dtype,
                               const rs_solver_opts *opts, rs_solver **out);
void rs_eigensolve_destroy(rs_solver *s);

/* One step on psi (DEVICE [nblk][np][B], the first nstates states
 * orthonormal and the padding states zero on entry; updated in place).  eig and resnorm (HOST double [nstates], may be NULL) receive
 * the step's Rayleigh-Ritz eigenvalues and residual norms; *nconv (HOST, may
 * be NULL) the number of states with resnorm < tol.  Synchronises the stream
 * once.  Errors: RS_ENOTPOSDEF if the final orthonormalisation fails,
 * RS_ENONFINITE if an eigenvalue or residual is not finite. */
rs_status rs_eigensolve_step(rs_solver *s, void *psi, double *eig, double *resnorm,
                             int32_t *nconv, void *stream);

/* Orthonormalises the solver's states in psi (eq. (8), as at the end of a
 * step), leaving the padding states of a partial last block zero: the
 * starting point of rs_eigensolve_step.  Synchronises.  RS_ENOTPOSDEF when
 * the states are linearly dependent. */
rs_status rs_eigensolve_orthonormalize(rs_solver *s, void *psi, void *stream);

/* ------------------------------------------------- SCF loop, Sec. 3
 * Fig. "groundstate": per iteration V_eff = V_ion + V_H[n_in] + V_xc[n_in]
 * (V_H by the FFT solve above; V_xc the local density approximation: Dirac
 * exchange and the Perdew-Zunger (1981) correlation, unpolarised), then
 * eig_steps rs_eigensolve_step calls on the states with that potential,
 * then n_out = 2 sum_{k < nocc} psi_k^2 (eq. 1b; closed shell, real
 * states) and F = n_out - n_in, and Broyden's second method in Anderson's
 * form: with the differences dn_j, dF_j of the last `history` iterations,
 * gamma solves (dF_i . dF_j) gamma = (dF_i . F) (h^3-weighted; gamma = 0 if
 * singular) and n_in <- n_in + mix F - sum_j gamma_j (dn_j + mix dF_j).
 * Densities, potentials and the history are FP64; the states are dtype. */
typedef struct {
    int32_t nocc;         /* occupied states (2 electrons each), 1..nstates */
    int32_t eig_steps;    /* eigensolver steps per SCF iteration, 1..100    */
    int32_t history;      /* mixing history length, 0..8                    */
    double  mix;          /* mixing weight, (0, 1]                          */
    rs_solver_opts solver;  /* options of the eigensolver it runs          */
} rs_scf_opts;
typedef struct rs_scf rs_scf;
/* vion: DEVICE double [np], copied.  Creates its eigensolver (whose local
 * potential is the handle's V_eff) and its Hartree solver; finite grids
 * only. */
rs_status rs_scf_create(const rs_grid *g, const rs_nl *nl, const double *vion, int32_t nstates,
                        int32_t B, int32_t dtype, const rs_scf_opts *opts, rs_scf **out);
void rs_scf_destroy(rs_scf *s);
/* Orthonormalises psi (the eigensolver's layout) and takes its density as
 * the first n_in.  Synchronises. */
rs_status rs_scf_start(rs_scf *s, void *psi, void *stream);
/* One SCF iteration on psi (updated in place).  eig, resnorm: HOST double
 * [nstates] (may be NULL), the last eigensolver step's outputs; dens_res:
 * HOST, ||n_out - n_in|| = (h^3 sum F^2)^(1/2) of this iteration (before
 * mixing).  Synchronises. */
rs_status rs_scf_iterate(rs_scf *s, void *psi, double *eig, double *resnorm, double *dens_res,
                         void *stream);
/* Copies of the current input density (after the last mixing) and of the
 * last output density into DEVICE double [np] buffers (either may be
 * NULL).  Asynchronous. */
rs_status rs_scf_density(const rs_scf *s, double *n_in, double *n_out, void *stream);

/* ------------------------------------------- learned preconditioner
 * Not from the paper: its RMM-DIIS step (Sec. 3) leaves the preconditioner
 * open and uses a filter; this replaces the filter by a small network
 * trained on the shifted kinetic problem.
 *
 * Network f: three 3x3x3 cross-correlation layers without bias, channels
 * 1 -> 8 -> 8 -> 1, tanh after the first two; every layer's output is zero
 * off the domain.  Preconditioner for a residual r of a state with shift
 * sigma < 0:  K(r) = s g(sigma) f(r / s), s = rms of r over the grid points,
 * g = softplus(a + b log(-sigma h^2)); K(0) = 0.  Parameters: one FP32
 * vector of RS_CNN_NPARAM values, w1 [8][1][27], w2 [8][8][27],
 * w3 [1][8][27] (weight layout [out][in][tap], tap t = 9 dz + 3 dy + dx
 * reads the input at offset (dx-1, dy-1, dz-1)), then a, b.
 * Network fields are dense boxes [n][Z][Y][X] (FP32, DEVICE, x fastest);
 * on a grid the box is the smallest axis-aligned box holding every point,
 * zero outside the domain, wrapped on periodic grids.  Network arithmetic
 * is FP32. */
#define RS_CNN_NPARAM 2162
typedef struct rs_cnn rs_cnn;

/* Scratch for batches of up to max_batch boxes of up to max_box points
 * (max_batch * max_box <= 2^28); about 17 * 4 bytes per point for
 * inference, twice that once training starts.  Parameters start at 0. */
rs_status rs_cnn_create(int32_t max_batch, int64_t max_box, rs_cnn **out);
void rs_cnn_destroy(rs_cnn *c);
/* HOST float [RS_CNN_NPARAM]; setting also resets the Adam moments. */
rs_status rs_cnn_set_params(rs_cnn *c, const float *params);
rs_status rs_cnn_get_params(const rs_cnn *c, float *params);
/* Checkpoint of the network's training state: the parameters, both Adam
 * moments and the Adam step count, written to / read from the file at path
 * (binary: an 8-byte tag "RSCNN001", int64 parameter count, int64 step
 * count, then 3 * RS_CNN_NPARAM floats, little endian).  Loading restores
 * the state exactly, so training resumes where it stopped.  RS_EINVAL when
 * the file cannot be opened, is short, or holds another layout.
 * Synchronous. */
rs_status rs_cnn_save(const rs_cnn *c, const char *path);
rs_status rs_cnn_load(rs_cnn *c, const char *path);

/* f = network(u) for n boxes of dims {Z, Y, X}, no mask (all points
 * inside), zero outside the box or wrapped (periodic != 0).
 * Asynchronous. */
rs_status rs_cnn_forward(rs_cnn *c, const float *u, float *f, int32_t n,
                         const int32_t dims[3], int32_t periodic, void *stream);

/* Training loss and gradient on a batch of crops u (network input r/s),
 * t (target x/s), shifts sigma (DEVICE double [n], < 0), zero outside each
 * crop.  The error is measured in the energy norm of A_i = T - sigma_i
 * (T the 25-point stencil on the crop, zero outside):
 * loss = sum_i <e_i|A_i e_i> / sum_i <M t_i|A_i M t_i>,
 * e_i = M (g_i f(u_i) - t_i), M the points at least `margin` from the crop
 * faces.  The gradient (all RS_CNN_NPARAM
 * values, FP32 with FP64 sums over points) is kept for rs_cnn_adam_step and
 * copied to grad (HOST, may be NULL); du (DEVICE [n][Z][Y][X], may be NULL)
 * receives dloss/du.  Synchronises when loss or grad is given. */
rs_status rs_cnn_loss_grad(rs_cnn *c, const float *u, const float *t, const double *sigma,
                           int32_t n, const int32_t dims[3], double h, int32_t margin,
                           double *loss, float *grad, float *du, void *stream);

/* One Adam update (Kingma and Ba, 2015) of the parameters with the last
 * gradient: m = b1 m + (1-b1) g, v = b2 v + (1-b2) g^2,
 * p -= lr (m / (1-b1^t)) / (sqrt(v / (1-b2^t)) + eps).  Asynchronous. */
rs_status rs_cnn_adam_step(rs_cnn *c, float lr, float beta1, float beta2, float eps,
                           void *stream);

/* out = K(r) for fields r, out [nblk][np][B] of dtype (DEVICE, distinct);
 * sigma DEVICE double [nblk*B].  The grid's box must fit max_box and B
 * must not exceed max_batch.  Asynchronous. */
rs_status rs_cnn_precondition(rs_cnn *c, const rs_grid *g, const void *r, const double *sigma,
                              void *out, int32_t nblk, int32_t B, int32_t dtype, void *stream);

/* Dims {Z, Y, X} of the grid's box. */
rs_status rs_cnn_box(rs_cnn *c, const rs_grid *g, int32_t dims[3]);

/* Training crops: for crop i with desc (HOST int32 [ncrops][4]) = (state k,
 * box origin x0, y0, z0), u_i = r_k / s_k and t_i = x_k / s_k on the crop's
 * points (dims cdims {Z, Y, X}), s_k the rms of r_k over the grid; zero off
 * the domain, wrapped on periodic grids.  Synchronises. */
rs_status rs_cnn_crops(rs_cnn *c, const rs_grid *g, const void *r, const void *x, int32_t nblk,
                       int32_t B, int32_t dtype, int32_t ncrops, const int32_t *desc,
                       const int32_t cdims[3], float *u_out, float *t_out, void *stream);

/* Training targets: x_k = (T - sigma_k)^-1 r_k with T the kinetic stencil
 * (Sec. 5.1) by conjugate gradients, each state to |r - (T - sigma) x| <=
 * tol |r|; sigma DEVICE double [nblk*B], each < 0 (so T - sigma is positive
 * definite).  r, x [nblk][np][B] of dtype, distinct.  Allocates its scratch
 * (3 fields).  *iters (HOST, may be NULL) = iterations used.  Synchronises
 * every 10 iterations.  RS_ENOTCONV if maxit is reached first. */
rs_status rs_shifted_solve(const rs_grid *g, const void *r, const double *sigma, void *x,
                           int32_t nblk, int32_t B, int32_t dtype, double tol, int32_t maxit,
                           int32_t *iters, void *stream);

/* Use the network as a second preconditioner of the solver (NULL: the
 * filter alone).  Each step then also applies the kinetic stencil to psi for
 * the shifts sigma_k = -<psi_k|T|psi_k>, and per active state the trial step
 * minimises the Rayleigh quotient over span{psi, d_f, d_n}, d_f = K_f R0
 * (filter) and d_n = K_n R0 (network): the lowest eigenvector of that 3x3
 * generalised problem (first component one) gives the coefficients (a, b)
 * of K = a K_f + b K_n, which is the state's preconditioner for the rest of
 * the step (lambda = 1).  The filter thus stays in every trial subspace and
 * judges the network state by state and step by step: a useless network
 * gets b ~ 0.  When the 3x3 problem is singular (d_n zero, not finite or
 * parallel to d_f) the state takes the filter step (b = 0).  Costs per step
 * one more H application (H d_n) and m network applications.  Allocates two
 * field arrays on first use.  The handle must outlive its use. */
rs_status rs_eigensolve_set_precond(rs_solver *s, rs_cnn *c);

/* Counters of the last rs_eigensolve_step. */
typedef struct {
    int32_t steps;          /* steps taken by this solver                      */
    int32_t rr_sweeps;      /* Jacobi sweeps of its Rayleigh-Ritz problem      */
    int32_t frozen_blocks;  /* blocks frozen by the stopping rule              */
    int32_t net_states;     /* states whose trial step gave the network a
                               nonzero coefficient (0 with the filter alone)   */
} rs_solver_stats;
rs_status rs_eigensolve_stats(const rs_solver *s, rs_solver_stats *out);

/* With opts.record: the last step's residuals R0 (after Rayleigh-Ritz) and
 * shifts sigma_k = -<psi_k|T|psi_k> into R (DEVICE, the psi layout) and
 * sigma (DEVICE double [nblk * B]; 0 for padding states).  Asynchronous. */
rs_status rs_eigensolve_residuals(rs_solver *s, void *R, double *sigma, void *stream);

#ifdef __cplusplus
}
#endif
#endif /* RSDFT_H */
