/*
 * aimm: the solve-time path of the macromodel surface-integral-equation method for
 * large arrays of scatterers (Patel, Triverio, Hum, arXiv:1712.02443), on AMD
 * Instinct MI355X (gfx950).
 *
 * The library solves the final system of section IV, eq. finalsystem,
 *     (D - G T A^-1 B) E = V,
 * by GMRES (section V), and applies its matrix-vector product, eq. MV_product1,
 *     y = (D - G T A^-1 B) x,
 * with G accelerated by the adaptive integral method (section V, steps (i)-(iii)).
 *
 * Model of the problem (section III): an array of px x py elements on a square
 * lattice, every element enclosed by the same closed equivalent surface (one RWG
 * mesh, N RWG functions), each element of one of n_types distinct kinds.  The block
 * T_m A_m^-1 B_m is shared by all elements of one kind (section III: computed once
 * per distinct element) and is given to the library as one dense N x N block M_t.
 * D is block diagonal with one sparse N x N block shared by all elements (the
 * surface is the same for all of them).  The library computes everything else:
 * AIM stencils and projection weights, the Green's-function spectrum, the exact
 * near-field Galerkin entries of eq. Gouter1 and their pre-correction.
 *
 * Conventions
 *   - Complex numbers are interleaved (re, im).  AIM_FP64 data is complex128,
 *     AIM_MIXED data is complex64.  Right-hand sides and solutions of gmres_solve
 *     are always complex128.
 *   - Unknowns are element-major: index r * (n_elem * N) + m * N + n for right-hand
 *     side r, element m = iy * px + ix, RWG function n.
 *   - Lengths are in wavelengths; element m is centred at (pitch_cells * h * ix,
 *     pitch_cells * h * iy, 0); the surface mesh is given in element-local
 *     coordinates.
 *   - Pointers named "device" must be device memory owned by the caller; the
 *     library never frees them.  Host pointers are read during the call only.
 *   - Streams are hipStream_t passed as void* (NULL = the null stream).  One op is
 *     used by one stream at a time; calls on different ops may overlap.
 *   - Every entry point returns an aim_status.  On AIM_EINVAL no output is
 *     touched; aim_last_error() returns a thread-local message for the last failure.
 */
#ifndef AIMM_H
#define AIMM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct aim_op aim_op;

enum aim_status {
  AIM_OK = 0,
  AIM_ENOCONV = 1,   /* gmres_solve: some right-hand side did not reach tol */
  AIM_EINVAL = -1,   /* bad argument; nothing was modified */
  AIM_ENOMEM = -2,   /* device allocation failed */
  AIM_EDEVICE = -3,  /* a HIP call or kernel launch failed */
  AIM_ESTATE = -4    /* operator data missing (macromodels or D not set) */
};

enum aim_precision {
  AIM_FP64 = 0,  /* every step in complex FP64 */
  AIM_MIXED = 1  /* complex FP32 storage and arithmetic for the product */
};

enum aim_matvec_flags {
  AIM_FULL = 0,      /* y = D x - G (M x)                                  */
  AIM_G_ONLY = 1,    /* y = G x: AIM far field plus pre-corrected near field */
  AIM_FAR_ONLY = 2   /* y = sum_psi I_psi H_psi P_psi x (grid part only)     */
};

/* One closed equivalent surface in element-local coordinates (section II-A). */
typedef struct {
  int32_t n_vert, n_tri, n_rwg;
  const double* vert;   /* host [n_vert][3] */
  const int32_t* tri;   /* host [n_tri][3], counter-clockwise seen from outside */
  const int32_t* rwg;   /* host [n_rwg][4] = v_a, v_b (the edge), T+, T- */
} aim_surface;

/* The array and the AIM parameters (sections III and V). */
typedef struct {
  double k;             /* wavenumber (2 pi in wavelength units) */
  double eta;           /* free-space impedance */
  double h;             /* AIM grid spacing */
  double r_near;        /* near-field radius between RWG edge midpoints */
  int32_t order;        /* stencil order N_O (N_O + 1 nodes per axis), 1..3 */
  int32_t px, py;       /* lattice size */
  int32_t pitch_cells;  /* lattice pitch in grid cells */
  int32_t n_types;      /* number of distinct elements */
  const int32_t* elem_type;  /* host [py*px], values in [0, n_types) */
  int32_t max_rhs;      /* largest right-hand-side count any call will use */
} aim_array;

typedef struct {
  int32_t n_rwg, n_elem, n_types;
  int32_t nx, ny, nz;          /* unpadded AIM grid (nodes) */
  int32_t lx, ly;              /* padded FFT lengths along x and y */
  int32_t n_offsets;           /* lattice offsets with near-field pairs */
  int64_t near_nnz;            /* pre-corrected near-field entries per element row block */
  int64_t d_nnz;               /* entries of the D block (0 until set) */
  int64_t device_bytes;        /* device memory held by the op */
  int32_t paths;               /* kernels in use: AIM_PATH_FFT_REGISTER (FFT passes of
                                  in-register DFTs, else radix stages), AIM_PATH_NEAR_MFMA
                                  (near field on the matrix cores, else sparse rows),
                                  AIM_PATH_GEMM_BF16X3 (mixed-path macromodel product as
                                  split-BF16 MFMA with FP32 accumulation, else FP32 MFMA);
                                  0 for host-only ops */
} aim_info;

#define AIM_PATH_FFT_REGISTER 1
#define AIM_PATH_NEAR_MFMA 2
#define AIM_PATH_GEMM_BF16X3 4

/* Build the AIM operator of section V for the array: stencils, projection and
 * interpolation weights, FFT plan and Green's-function spectrum (on the device),
 * and the pre-corrected near field (exact entries of eq. Gouter1 on near pairs minus
 * their grid approximation).  Allocates device memory for max_rhs right-hand sides.
 * Uses the current HIP device; uploads and the spectrum kernels run on `stream`, which
 * is synchronised before the call returns.  *out is set only on success. */
int aim_build_grid(const aim_surface* surface, const aim_array* array, void* stream, aim_op** out);

/* Launch configuration of the product's kernels (what a tuner chooses; the results of
 * every choice agree to rounding).  Fields of 0 (fft_b, interp tile) or -1 (flags) keep
 * the current value in aim_set_tuning. */
typedef struct {
  int32_t fft_b[2];      /* ky lines per x-pass workgroup, [AIM_FP64, AIM_MIXED]: must divide
                            the padded y length and fit one workgroup's LDS */
  int32_t interp_tx, interp_ty;  /* elements per interpolation workgroup, tx ty <= 4; refused
                                    if the tile's potentials do not fit one workgroup's LDS in
                                    complex64, lowered at launch where they do not in complex128 */
  int32_t gemm_bf16;     /* mixed-path macromodel product: 1 split-BF16 MFMA (needs N % 8 == 0),
                            0 FP32 MFMA */
  int32_t fft_register;  /* 1 four-step passes of in-register DFTs (where compiled), 0 radix stages */
  int32_t near_block[2]; /* near field on the matrix cores, [AIM_FP64, AIM_MIXED]: blocks of 16
                            elements per workgroup, 1 or 2 (two share every coefficient load) */
  int32_t near_fork[2];  /* where the near field leaves the caller's stream for the op's second
                            stream, [AIM_FP64, AIM_MIXED]: 0 after the macromodel product, 1 after
                            the projection, 2 after the y FFT pass (-1 keeps the current value) */
} aim_tuning;

/* Current launch configuration of the op. */
int aim_get_tuning(const aim_op* op, aim_tuning* tuning);

/* Set the launch configuration (AIM_EINVAL for a value the op cannot run, nothing changed).
 * Takes effect from the next call; the op must have no work in flight. */
int aim_set_tuning(aim_op* op, const aim_tuning* tuning);

/* Change the kind of every element (host [py*px], values in [0, n_types)) of a built op,
 * keeping its grid, Green's-function spectrum, near field, macromodels, D and
 * preconditioner blocks, which do not depend on where each kind sits (section III: the
 * blocks are per distinct element).  For serving many arrays of one size with one op.
 * The op must have no work in flight on any stream; the copy runs on `stream`, which is
 * synchronised before the call returns. */
int aim_set_elem_type(aim_op* op, const int32_t* elem_type, void* stream);

/* The host part of aim_build_grid alone: stencils, weights and the pre-corrected
 * near field, with no device call.  The op serves aim_get_info, aim_get_near and
 * the host parts of aim_set_macromodels, aim_set_dmatrix, aim_build_preconditioner
 * and aim_get_preconditioner; every device entry point returns AIM_ESTATE on it.
 * For inspection and tests on hosts without a GPU. */
int aim_build_host(const aim_surface* surface, const aim_array* array, aim_op** out);

/* Per-kind block M_t = T_t A_t^-1 B_t (section III, eq. Tm1 and eq. JABE), host
 * complex128 [n_types][N][N], column-major within each block.  Copied (to the
 * device, and kept on the host for aim_build_preconditioner; a host-only op keeps
 * the host copy only).  May be called again to replace the blocks. */
int aim_set_macromodels(aim_op* op, const double* M);

/* The sparse block D_m (section IV) shared by all elements, as host coordinate
 * lists: rows[nnz], cols[nnz] in [0, N), vals complex128 [nnz].  Copied (host copy
 * kept as for the macromodels).  Set once per op (AIM_ESTATE on a second call). */
int aim_set_dmatrix(aim_op* op, int64_t nnz, const int32_t* rows, const int32_t* cols,
                    const double* vals);

/* u = blockdiag(M_t(m)) x for nrhs right-hand sides (section III).  x, u: device. */
int macro_apply(aim_op* op, const void* x, void* u, int32_t nrhs, int32_t precision,
                void* stream);

/* The product of eq. MV_product1, or a part of it (see aim_matvec_flags).
 * x, y: device, nrhs <= max_rhs.  No allocation and no host synchronisation. */
int aim_matvec(aim_op* op, const void* x, void* y, int32_t nrhs, int32_t precision,
               int32_t flags, void* stream);

/* Kernel timing of the full product with HIP events on `stream`: after one full
 * product, each kernel is launched once untimed and then reps times back to back
 * between two events; ms[k] receives the mean duration in milliseconds of kernel k:
 * 0 macromodel GEMM, 1 projection (step (i)), 2 forward FFT along y, 3 FFT along x
 * with the kernel-spectrum product, 4 inverse FFT along y (step (ii)), 5 pre-corrected
 * near field, 6 interpolation (step (iii)) fused with D and the final combination.
 * The x pass writes to a temporary device buffer of the spectrum pass size (allocated
 * and freed inside the call; AIM_ENOMEM if that fails).  y holds the product on return.
 * ms: host [7].  Synchronises the stream. */
int aim_time_kernels(aim_op* op, const void* x, void* y, int32_t nrhs, int32_t precision,
                     int32_t reps, double* ms, void* stream);

/* Step (i) alone: grid charges and currents Q[r][psi][x][y][z] (psi = x, y, z, phi)
 * on the unpadded grid.  u: device vector, Q: device [nrhs][4][nx][ny][nz]. */
int aim_project(aim_op* op, const void* u, void* Q, int32_t nrhs, int32_t precision,
                void* stream);

/* Step (ii) alone: grid potentials Phi = H Q (aperiodic convolution with the sampled
 * Green's function).  Q and Phi: device [nrhs][4][nx][ny][nz]; may alias. */
int aim_convolve(aim_op* op, const void* Q, void* Phi, int32_t nrhs, int32_t precision,
                 void* stream);

/* Plane-wave excitation of eq. V1, V_n = -<Lambda_n, E_inc>, for incidence angles
 * (theta, phi) in radians and polarisation pol (0 = theta-hat, 1 = phi-hat).
 * theta, phi, pol: host [nrhs].  b: device complex128. */
int aim_plane_wave_rhs(aim_op* op, const double* theta, const double* phi, const int32_t* pol,
                       int32_t nrhs, void* b, void* stream);

typedef struct {
  int32_t restart;      /* Krylov dimension per cycle (GMRES(m)) */
  int32_t max_iters;    /* total inner iterations per right-hand side */
  int32_t precision;    /* AIM_FP64: all FP64.  AIM_MIXED: inner cycles with FP32
                           products and FP32 basis storage, FP64 dot products,
                           Hessenberg and Givens; FP64 residual at every restart */
  int32_t x0_given;     /* 0: start from x = 0; 1: start from the x passed in */
  int32_t check_every;  /* most iterations between host checks of the stop flags
                           (>= 1); checks come earlier where the residual estimate
                           predicts convergence.  Results do not depend on it. */
  int32_t precond;      /* aim_precond: AIM_PRECOND_NONE, or AIM_PRECOND_BLOCK_JACOBI
                           (right preconditioning, A P z = b, x = P z, with the
                           blocks of aim_build_preconditioner; the residual that
                           tol and the stats refer to is still b - A x) */
  int32_t system;       /* AIM_FULL: A = D - G M, the final system (eq. finalsystem);
                           AIM_G_ONLY: A = G, the EFIE of the surfaces themselves
                           (standard MoM on scatterer meshes: no macromodels or D
                           needed; block-Jacobi then wants blocks built with
                           M_t = -I and an empty D, which make them G_self^-1) */
  int32_t graphs;       /* 1: each inner iteration's launches are captured once per
                           iteration index as a HIP graph (on a library stream) and
                           replayed on the caller's stream in later cycles and solves;
                           the graphs stay with the op until its Krylov workspace, launch
                           configuration or element kinds change.  0: launched one by
                           one.  Results are bit-identical either way. */
  double tol;           /* relative residual target ||b - A x|| / ||b|| */
} gmres_opts;

enum aim_precond {
  AIM_PRECOND_NONE = 0,
  AIM_PRECOND_BLOCK_JACOBI = 1
};

typedef struct {
  int32_t iters;        /* inner iterations */
  int32_t restarts;     /* completed cycles */
  int32_t converged;    /* 1 if the FP64 true relative residual <= tol */
  int32_t matvecs;      /* products applied to this right-hand side (the first
                           cycle from x = 0 needs none for its residual) */
  double true_relres;   /* final FP64 true relative residual */
} gmres_stat;

/* Solve eq. finalsystem for nrhs right-hand sides with restarted GMRES (section V),
 * one independent Krylov space per right-hand side.  b, x: device complex128
 * [nrhs][n_unknowns]; stats: host [nrhs].  Returns AIM_ENOCONV (and the last
 * iterate in x) if a right-hand side misses tol within max_iters.  Allocates the
 * Krylov basis on first use and keeps it with the op. */
int gmres_solve(aim_op* op, const void* b, void* x, int32_t nrhs, const gmres_opts* opts,
                gmres_stat* stats, void* stream);

/* Block-Jacobi preconditioner of the final system (section IV eq. finalsystem;
 * the paper preconditions GMRES with an incomplete factorisation of the near-field
 * matrix, section VI).  The diagonal block of element m is D - G_self M_t(m), where
 * G_self is the AIM operator on one element's own RWG functions (the grid part on
 * every pair plus the pre-corrected near field of lattice offset (0, 0)); it is the
 * same for all elements of one kind, so the library computes one FP64 inverse
 * P_t = (D - G_self M_t)^-1 per kind on the host (partially pivoted LU) and keeps it
 * on the device in the layouts of M_t.  Needs aim_set_macromodels and
 * aim_set_dmatrix first (AIM_ESTATE otherwise); aim_set_macromodels makes it stale
 * until it is built again.  AIM_EINVAL if a block is singular.  Works on host-only
 * ops too (host copy only).  Runs for seconds on large N (O(N^3) per kind). */
int aim_build_preconditioner(aim_op* op);

/* Copy of the blocks P_t: host complex128 [n_types][N][N], column-major. */
int aim_get_preconditioner(const aim_op* op, double* P);

/* y = blockdiag(P_t(m)) x for nrhs right-hand sides; x, y: device, element-major,
 * must not alias.  The grouped product of macro_apply with the blocks P_t. */
int precond_apply(aim_op* op, const void* x, void* y, int32_t nrhs, int32_t precision, void* stream);

/* Far field of the solution's equivalent currents, for the radiation patterns and
 * bistatic RCS of section VI: with J = -M x (the equivalent currents J^ = T J =
 * -T A^-1 B E^ of eq. Toperator and eq. JABE; J = x when system is AIM_G_ONLY, the
 * surface currents of a standard MoM solve) and element m centred at c_m,
 *   E(r^) = -(j k eta / 4 pi) (I - r^ r^) . sum_m exp(j k r^ . c_m)
 *           sum_n J_{m,n} int Lambda_n(r) exp(j k r^ . r) dS,
 * the far-zone field E r exp(j k r) for unit incident amplitude, in FP64 (the sum over
 * elements runs as a complex GEMM on the FP64 matrix cores).  x: device complex128
 * [nrhs][n_unknowns] (a solution of gmres_solve); rhat: host [ndir][3] unit vectors;
 * E: device complex128 [nrhs][ndir][3]; rcs_db: device double [nrhs][ndir] receiving
 * 10 log10(4 pi |E|^2) (RCS in dB relative to a square wavelength), or NULL.  Needs
 * the macromodels for AIM_FULL (AIM_ESTATE otherwise).  Allocates a device workspace on first use
 * and when ndir grows, and keeps it with the op. */
int aim_far_field(aim_op* op, const void* x, int32_t nrhs, int32_t ndir, const double* rhat, void* E,
                  void* rcs_db, int32_t system, void* stream);

/* aim_far_field without any device allocation, for callers that cannot allocate (code
 * under HIP graph capture, serving loops with a fixed memory budget): the same kernels
 * and results, with the directions, phase tables and per-tile partials in a
 * library-owned scratch array of 16 MiB per GPU (held until the process ends) instead
 * of an op workspace.  The workspace a call needs is
 *   256-byte-rounded 24 ndir + 16 ndir (px + py) + 48 ceil(N / 32) nrhs ndir  bytes;
 * a call needing more returns AIM_EINVAL (nothing modified).  Every call on one GPU
 * shares that GPU's array: calls that overlap on one GPU (other streams, other ops,
 * other host threads) race and must be ordered by the caller.  The op's own device
 * buffers, allocated when it was built, serve as before.  Other arguments, errors and
 * results as aim_far_field. */
int aim_far_field_noalloc(aim_op* op, const void* x, int32_t nrhs, int32_t ndir, const double* rhat, void* E,
                          void* rcs_db, int32_t system, void* stream);

/* Macromodel generation (section II, section III) in the library, on the device, for
 * every element kind: scatterers[t] is the PEC surface of kind t (element-local
 * coordinates, inside the op's equivalent surface; RWG table as for aim_surface).  With
 * the op's surface as the equivalent surface S^ (n its inward normal) the library fills
 * the Galerkin blocks of eq. Gm_EJ_1 - Gm_EJ_3 and eq. G1 - G3 (L-type with the kernel's
 * static part in closed form; K-type with the Buffa-Christiansen dual functions on the
 * barycentric refinement of S^, principal value plus D / 2 on S^ itself), D of section
 * IV, then [T | Y] = G^(E^,H^)^-1 [G^(E^,J) | G^(E^,E^)], [A | B] = [G^(E,J) | G^(E,E^)] -
 * G^(E,H^) [T | Y] (eq. JM), R = A^-1 B and M = T R (eq. JABE, eq. Tm1) in FP64 by
 * Gauss-Jordan elimination and GEMMs on the matrix cores.  It then sets M (as
 * aim_set_macromodels) and D (as aim_set_dmatrix) on the op and keeps each kind's R on
 * the device for aim_recover_currents.  AIM_ESTATE if D is already set or the op is
 * host-only; AIM_EINVAL for a bad or open mesh or a singular block (an equivalent
 * surface at an interior resonance).  Synchronises the stream; allocates (and frees)
 * temporary device memory of about 144 n_tri^2 bytes for the largest mesh. */
int aim_build_macromodels(aim_op* op, const aim_surface* scatterers, void* stream);

/* Host copies of kind `kind`'s generated blocks: M complex128 [N][N], R = A^-1 B complex128
 * [N_t][N] (N_t = RWG functions of the kind's scatterer), D real [N][N], all column-major;
 * any output may be NULL.  AIM_ESTATE unless aim_build_macromodels succeeded on the op. */
int aim_get_macromodel(const aim_op* op, int32_t kind, double* M, double* R, double* D);

/* Scatterer unknowns: of kind `kind` (>= 0), or of the whole array (kind = -1, the sum
 * of the elements' N_t); -1 before aim_build_macromodels. */
int64_t aim_scatterer_unknowns(const aim_op* op, int32_t kind);

/* Current recovery on the original scatterers, J_m = -R_t(m) E^_m for every element m
 * (eq. JABE; the paper's inexpensive step after the solve), FP64, as grouped GEMMs on
 * the matrix cores.  x: device complex128 [nrhs][n_elem][N] (solutions of gmres_solve);
 * J: device complex128 [nrhs][aim_scatterer_unknowns(op, -1)], element-major with
 * element m's N_t(m) values after those of elements 0..m-1.  Synchronises the stream. */
int aim_recover_currents(aim_op* op, const void* x, void* J, int32_t nrhs, void* stream);

/* Sizes of the op (host only, no device work). */
int aim_get_info(const aim_op* op, aim_info* info);

/* Copy the pre-corrected near-field entries (host outputs, each of length
 * info.near_nnz): row n, offset index o, column n', complex128 value.  The offset
 * (dx, dy) of index o is returned in offsets[2*o], offsets[2*o+1]. */
int aim_get_near(const aim_op* op, int32_t* rows, int32_t* offs, int32_t* cols, double* vals,
                 int32_t* offsets);

/* Device bytes an op of this array would hold, Krylov basis included, for admission
 * decisions; host only.  Not included: the block-Jacobi blocks (aim_build_preconditioner,
 * about 3 n_types N^2 x 16 bytes) and the far-field workspace, allocated when first used. */
size_t aim_footprint_bytes(const aim_surface* surface, const aim_array* array, int32_t nrhs,
                           int32_t restart, int32_t precision);

/* Release every resource of the op (synchronises the device). NULL is ignored. */
void aim_destroy(aim_op* op);

/* Message of the last failing call on this thread ("" if none). */
const char* aim_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* AIMM_H */
