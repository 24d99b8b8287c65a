/*
 * lsh.h -- Lippmann-Schwinger homogenisation on the pattern P(M), MI355X (gfx950).
 *
 * C ABI of liblsh.so.  The library solves the discretised Lippmann-Schwinger
 * equation of Bergmann & Merkert, "FFT-based homogenization on periodic
 * anisotropic translation invariant spaces" (arXiv 1701.04685),
 * Thm. (pde_discretization), eq. (pde_coefficients):
 *
 *     E_y + Gamma^p_y (C(y) - C0) : (E_y + eps0) = 0,      y in P(M),
 *
 * with the fixed-point iteration of Moulinec and Suquet ("Basic Scheme",
 * Sec. 4) and returns the effective stress C^eff : eps0 (Sec. 3.1).
 *
 * Conventions (all entry points)
 *  - Every function returns an lsh_status; nothing throws across the ABI.
 *    On error, lsh_last_error() returns a thread-local message.
 *  - Host arrays passed in are copied; the caller keeps ownership.
 *  - Device memory is always allocated by the caller (for example as a torch
 *    uint8 tensor) and must outlive the work queued on `stream`.  The library
 *    itself never allocates device memory.
 *  - `stream` is a hipStream_t passed as void* (NULL = the default stream).
 *  - Voigt order is (11, 22, 33, 23, 13, 12).  Strains use engineering shear
 *    (gamma_23 = 2 eps_23); stresses and stiffness matrices are tensor
 *    components.  Internally the library works in Mandel form.
 *  - Real-space device fields are laid out [load][component][a1][a2][a3] with
 *    a = (a1, a2, a3) the SNF grid index of the point (lsh_pattern_points),
 *    a3 fastest.
 *  - Two-dimensional patterns (d = 2, the setting of the numerics of Sec. 4):
 *    strains, stresses and stiffness matrices are 2-D Voigt, order (11, 22, 12)
 *    (3 entries per strain or stress, 3x3 per stiffness), in plane strain.  The
 *    library holds such a pattern as the three-dimensional blockdiag(M, 1), whose
 *    frequencies all have k3 = 0; every 3-entry array below takes the place of
 *    the 6-entry one, and device fields carry 3 components.
 */
#ifndef LSH_H
#define LSH_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lsh_pattern lsh_pattern; /* opaque; created/destroyed by the library */

typedef enum {
  LSH_OK = 0,
  LSH_EINVAL = -1,        /* bad argument (null pointer, size, range)                        */
  LSH_ESINGULAR = -2,     /* det M == 0: P(M) needs a regular M (Sec. 2.1)                   */
  LSH_ENOINTERP = -3,     /* a bracket sum of |c_k(f)|^2 vanishes: translates not linearly
                             independent (Lemma (FI:Props) a/b)                              */
  LSH_ENOTELLIPTIC = -4,  /* a stiffness is not symmetric positive definite (Sec. 3.1)       */
  LSH_ENOTCONVERGED = -5, /* max_iter reached before the Cauchy residual met tol             */
  LSH_ENONFINITE = -6,    /* NaN/Inf in the iteration                                        */
  LSH_EDEVICE = -7,       /* a HIP runtime call failed                                       */
  LSH_EWORKSPACE = -8,    /* device buffer smaller than the *_bytes query returned           */
  LSH_EUNSUPPORTED = -9,  /* SNF factor or size outside what the GPU path supports           */
  LSH_ESTATE = -10        /* call order: kernel/stiffness not set or device data not bound  */
} lsh_status;

typedef enum {
  LSH_DIRICHLET = 0,          /* D_M, g = 1 on [-1/2,1/2)^d (Sec. 2.2, Def. (dlVP) remark)   */
  LSH_DIRICHLET_MODIFIED = 1, /* f_{M,0}: limit alpha -> 0 of the dlVP means (Sec. 2.2)       */
  LSH_DLVP = 2,               /* de la Vallee Poussin mean f_{M,g_alpha}, Def. (dlVP)          */
  LSH_BOXSPLINE = 3           /* periodised pattern Box spline f_{M,Xi} (Sec. 2.2)             */
} lsh_kernel;

typedef enum {
  LSH_FP64 = 0,      /* every step in double precision                                       */
  LSH_FP32_MIXED = 1 /* FFT, Green multiply and stress in float; residual norms, the
                        effective-stress average and Gamma^p alias sums in double            */
} lsh_precision;

typedef struct {
  int32_t iterations; /* Basic Scheme iterations performed for this load case              */
  int32_t converged;  /* 1 if the Cauchy residual reached tol                              */
  double residual;    /* last Cauchy residual ||E^k - E^{k-1}|| / ||E^k + eps0||            */
  double seconds;     /* wall time of the whole iteration loop (same for all loads)         */
} lsh_stats;

/* ------------------------------------------------------------------ pattern ---
 * Sec. 2.1: the lattice Lambda(M) = M^{-1} Z^d, the pattern P(M) (points in
 * [-1/2,1/2)^d) and the generating set G(M^T); m = |det M|.  The library
 * takes the integer Smith normal form M = U diag(e1,e2,e3) V and orders P(M)
 * by a in Z_e1 x Z_e2 x Z_e3 (y = M^{-1} U a mod 1) and G(M^T) by b
 * (h = V^T b mod M^T); the pattern DFT of eq. (Fouriermatrix) is then the
 * plain 3-D DFT over that grid.
 *   d      : 3, or 2 for a pattern of the plane (held as blockdiag(M, 1): its
 *            SNF has e1 = 1 and its points have y3 = 0).
 *   M      : d*d integers, row-major.
 *   out    : receives a new pattern; release with lsh_destroy.
 * Errors: LSH_EINVAL (d not 2 or 3, null), LSH_ESINGULAR (det M == 0),
 *         LSH_EUNSUPPORTED (|det M| beyond int32 grid limits, or entries so large
 *         that the exact integer SNF would overflow int64).                        */
int lsh_create_pattern(int d, const int64_t *M, lsh_pattern **out);
void lsh_destroy(lsh_pattern *p);

/* m = |det M| and the SNF diagonal e (e1 | e2 | e3) of the three-dimensional
 * pattern the library holds (for d = 2 that of blockdiag(M, 1)).                 */
int lsh_pattern_info(const lsh_pattern *p, int64_t *m, int64_t e[3]);

/* The unimodular SNF factors, M = U diag(e) V, each 3x3 row-major.                */
int lsh_pattern_snf(const lsh_pattern *p, int64_t U[9], int64_t V[9]);

/* The points of P(M) in storage order: y = y_num / m, y in [-1/2,1/2)^d exactly.
 *   y_num : host int64 array of m*d entries, caller-allocated.                    */
int lsh_pattern_points(const lsh_pattern *p, int64_t *y_num);

/* -------------------------------------------------------- generating function ---
 * Chooses f, and with it the periodised Green operator of
 * Def. (gamma_tilde_fourier), Gamma^p_h = m [ {Gamma0_k |c_k(f)|^2} ]^M_h, for
 * orthonormalised translates (Lemma (FI:Props) c):
 *   Gamma^p_h = sum_z g(x+z)^2 Gamma0_{h+M^T z} / sum_z g(x+z)^2,  x = M^{-T} h.
 *   LSH_DIRICHLET, LSH_DIRICHLET_MODIFIED : nparams = 0.
 *   LSH_DLVP      : params = alpha[d], each in [0, 1], the trapezoid of Sec. 2.2
 *                   (g_alpha = B_Xi, Xi = (diag alpha, I); alpha = 1 is Fejer).
 *   LSH_BOXSPLINE : params = {s, Xi[d*s] (columns, pattern coordinates, row-major
 *                   d x s, spanning R^d), R, tail}; the alias sum runs over z in
 *                   [-R,R]^d (Sec. 4.2 truncates the bracket sums to a box of
 *                   terms; R defaults to 16).  tail = 1 adds the aliases beyond R
 *                   along the slow axes (one direction with a +-1 entry there,
 *                   all others 0): their weight is the mass the identity
 *                   sum_n sinc^2(pi (c + n)) = 1 leaves outside, their Green
 *                   operator that of M^T e_i; the truncation error then falls
 *                   like R^-3 instead of 1/R.  s <= 16 (d = 3), <= 15 (d = 2).
 * Host only.  Errors: LSH_EINVAL (kind, parameter count or range).               */
int lsh_set_kernel(lsh_pattern *p, lsh_kernel kind, const double *params, int nparams);

/* ------------------------------------------------------------------ stiffness ---
 * The piecewise-constant stiffness C(y) (Def. (weak_pde)) and the reference C0
 * of the Green operator (Def. (projection)).
 *   nphase   : 1..256 phases.
 *   C_voigt  : nphase*36 doubles, Voigt 6x6 per phase (row-major); d = 2:
 *              nphase*9, Voigt 3x3 (11, 22, 12).
 *   C0_voigt : 36 doubles (d = 2: 9).
 *   phase    : m bytes, phase index of each point in storage order.
 * d = 2: the 3x3 matrices are the in-plane blocks of plane-strain tensors; the
 * library completes them with out-of-plane entries shared by C0 and every
 * phase (those of the isotropic tensor with C0's Lame constants when C0 is
 * isotropic), so C - C0 acts in the plane only.
 * Host only (copied).  Errors: LSH_EINVAL, LSH_ENOTELLIPTIC (a matrix not SPD).  */
int lsh_set_stiffness(lsh_pattern *p, int nphase, const double *C_voigt,
                      const double *C0_voigt, const uint8_t *phase);

/* Discretisation solved by lsh_solve / lsh_solve_batch:
 *   LSH_SCHEME_LS (default): the Lippmann-Schwinger form, eq. (pde_coefficients),
 *     Thm. (pde_discretization), iterated in the polarisation form
 *       E <- -Gamma^p[(C - C0):(E + eps0)];
 *   LSH_SCHEME_VE: the variational form, eq. (pde_coefficients_variational),
 *     Thm. (ls_discretization), iterated in the strain-update form
 *       E <- E - Gamma^p[C:(E + eps0)].
 *   LSH_SCHEME_CG: conjugate gradients (the Krylov alternative named in Sec. 1)
 *     for the Dirichlet kernel on a pattern of odd m (no Nyquist faces).  There
 *     Gamma^p C0 projects onto the compatible strains, eq. (pde_coefficients) is
 *     equivalent to the variational system, and that system is symmetric
 *     positive definite in the C0 inner product.  Each iteration applies the
 *     operator once (the fixed-point schemes' unit of work; the count includes
 *     the start's application).  It stops on the Basic Scheme's Cauchy
 *     residual one fixed-point step from the current iterate,
 *     ||z|| / ||E + z + eps0|| with z = -Gamma^p C (E + eps0).  Same solution
 *     as LSH_SCHEME_LS; lsh_solve only (lsh_solve_batch refuses it).
 *     lsh_solve returns LSH_EUNSUPPORTED for other kernels or even m.
 *   LSH_SCHEME_LS_INC: the iterates of LSH_SCHEME_LS, computed from their
 *     increments.  The scheme is affine in E, so past the first iteration
 *       dE_{k+1} = -Gamma^p[(C - C0):dE_k],   E_{k+1} = E_k + dE_{k+1},
 *     with dE_{k+1} = E_{k+1} - E_k (eps0 drops out); the first iteration is
 *     the LS step.  In exact arithmetic the iterates, the residual history and
 *     the answer are LSH_SCHEME_LS's.  In rounded arithmetic the transforms
 *     act on the increment, so their rounding error scales with the increment
 *     rather than with the field, and the Cauchy residual ||dE|| / ||E|| keeps
 *     falling where the LS form levels off (about 1e-6 at contrast 100 in
 *     LSH_FP32_MIXED).  Same memory and passes as LS (the Green pass also
 *     writes the increment, one more field write per iteration).
 * LS and VE coincide for the Dirichlet kernel (Remark (constants)).  Changing
 * the scheme drops the device binding (call lsh_bind again).  Errors: LSH_EINVAL. */
typedef enum { LSH_SCHEME_LS = 0, LSH_SCHEME_VE = 1, LSH_SCHEME_CG = 2, LSH_SCHEME_LS_INC = 3 } lsh_scheme;
int lsh_set_scheme(lsh_pattern *p, lsh_scheme scheme);

/* ------------------------------------------------------------- device binding ---
 * Bytes of persistent device memory for this pattern at precision prec: the
 * phase map, FFT twiddles and the Green operator's table.  For LSH_BOXSPLINE,
 * and for the other smoothed kernels with an anisotropic C0, it holds the 21
 * entries of Gamma^p per half-spectrum bin; for the Dirichlet, modified
 * Dirichlet and dlVP kernels with an isotropic C0, the 15 fourth moments of
 * the alias directions per bin (the Dirichlet kernel with an anisotropic C0
 * needs none).  Sums in double, stored at prec; sized for the 21-entry table.
 * Needs lsh_set_kernel first.                                                     */
int lsh_persistent_bytes(const lsh_pattern *p, lsh_precision prec, size_t *bytes);

/* Uploads the phase map and twiddles into dev_persistent and builds the Green
 * operator's table on the GPU (synchronises `stream`; for the Box spline checks
 * every bracket sum is positive).  dev_persistent must stay alive while the
 * pattern is used at this precision.  Errors: LSH_ESTATE (kernel/stiffness not
 * set), LSH_EWORKSPACE, LSH_ENOINTERP, LSH_EUNSUPPORTED, LSH_EDEVICE.            */
int lsh_bind(lsh_pattern *p, lsh_precision prec, void *dev_persistent, size_t bytes,
             void *stream);

/* Evaluates the (Hermitian-symmetrised) Gamma^p at n frequency bins b
 * (3 ints each, 0 <= b1 <= e1/2, 0 <= b2 < e2, 0 <= b3 < e3) with the same
 * device code the solver uses; writes 21 doubles per bin (upper triangle of
 * the 6x6 Mandel matrix, row by row).  For d = 2 the bins and the matrix are
 * those of the three-dimensional pattern held (its in-plane block is the 2-D
 * operator).  dev_scratch: >= n*(24+21*8) bytes.
 * Synchronises `stream`.  For tests and diagnostics.                            */
int lsh_gamma_probe(const lsh_pattern *p, lsh_precision prec, const int64_t *bins, int n,
                    double *out, void *dev_scratch, size_t scratch_bytes, void *stream);

/* ---------------------------------------------------------------------- solve ---
 * Workspace bytes for lsh_solve with nload load cases at precision prec.          */
int lsh_solve_bytes(const lsh_pattern *p, int nload, lsh_precision prec, size_t *bytes);

/* Basic Scheme for eq. (pde_coefficients), Sec. 4:
 *   E^0 = 0 (or dev_E_init, mean removed);
 *   E^{k+1} = -F^{-1}[ Gamma^p_h F[(C - C0):(E^k + eps0)]_h ]   (real part);
 *   stop when ||E^{k+1} - E^k|| / ||E^{k+1} + eps0|| <= tol (Frobenius norms over
 *   all points; relative Cauchy criterion of Sec. 4).
 * Load cases run side by side and stop independently.
 *   nload        : 1..64 load cases.
 *   eps0_voigt   : host nload*6 macroscopic strains (Voigt, engineering shear);
 *                  nload*3 for d = 2 (as every per-load 6 below).
 *   tol          : Cauchy tolerance; tol < 0 runs exactly max_iter iterations
 *                  (fixed-count mode, returns LSH_OK).
 *   max_iter     : iteration limit, >= 1.
 *   dev_workspace: >= lsh_solve_bytes(...) bytes.
 *   dev_E_init   : optional device double [nload][6][m] start fluctuation (Voigt,
 *                  engineering shear) or NULL for zero; [nload][3][m] for d = 2.
 *   dev_E_out    : optional device double [nload][6][m] receiving the final E
 *                  ([nload][3][m] for d = 2).
 *   sigma_out    : host nload*6: sigma_bar = (1/m) sum_y C(y):(E_y + eps0)
 *                  (Voigt stress) at the final iterate (Sec. 3.1, C^eff : eps0).
 *   stats        : optional host nload entries.
 *   history      : optional host nload*max_iter residuals (NaN after stopping).
 * Runs on `stream` and synchronises it before returning.
 * Errors: LSH_ESTATE, LSH_EINVAL, LSH_EWORKSPACE, LSH_ENOTCONVERGED (outputs
 * still filled from the last iterate), LSH_ENONFINITE, LSH_EDEVICE.              */
int lsh_solve(lsh_pattern *p, int nload, const double *eps0_voigt, double tol, int max_iter,
              lsh_precision prec, void *dev_workspace, size_t ws_bytes, void *stream,
              const double *dev_E_init, double *dev_E_out, double *sigma_out,
              lsh_stats *stats, double *history);

/* ----------------------------------------------------- allocation-free solve ---
 * For callers that cannot allocate device memory (code running under HIP graph
 * capture of their own, tight serving loops, harnesses that forbid hipMalloc):
 * lsh_solve with the same arguments and results but no workspace argument.
 * The workspace lives in a fixed device array inside the library, of
 * LSH_NOALLOC_MAX_BYTES bytes, one per GPU the library runs on, held until the
 * process ends; its device address is looked up once per device.  The call
 * allocates nothing and instantiates no graph (its launches are issued one by
 * one), so it runs somewhat slower than lsh_solve for short problems.
 *   Limit: lsh_solve_bytes(p, nload, prec) <= LSH_NOALLOC_MAX_BYTES (64 MiB), e.g.
 *   32^3 with six loads in FP64, 48^3 with four loads in FP32; larger solves
 *   return LSH_EWORKSPACE with the bytes they need.
 *   Every call on one GPU shares that GPU's array and overwrites what the last
 *   call left there: calls that overlap on one GPU (other host threads, other
 *   streams) race, so the caller serialises them.  Everything a solve needs to
 *   start from zero is cleared by the call itself.
 * The pattern must be bound (lsh_bind) beforehand, which takes the caller's
 * persistent buffer.  Errors: as lsh_solve.                                        */
#define LSH_NOALLOC_MAX_BYTES (64u * 1024u * 1024u)
int lsh_solve_noalloc(lsh_pattern *p, int nload, const double *eps0_voigt, double tol, int max_iter,
                      lsh_precision prec, void *stream, const double *dev_E_init, double *dev_E_out,
                      double *sigma_out, lsh_stats *stats, double *history);

/* ------------------------------------------------------------------ autotuner ---
 * Each pass of an iteration has kernel variants (the axis-1 stress pass with or
 * without its middle stages fused in registers and its tile width along i3,
 * the axis-2 tile width, one or two load cases per Green-pass block).  lsh_autotune times every variant of
 * every pass on this pattern's own data (nload load cases, precision prec,
 * from a zero start; a warm-up launch, then the mean of three) with HIP events
 * on `stream`, and keeps the fastest for later lsh_solve and lsh_solve_batch
 * calls of this pattern (as a batch group's first pattern) at that precision.
 * Last it times the schedule: a whole four-pass iteration with the variants
 * just chosen (entry 0) against each variant of the two-pass iteration, which
 * splits the axis-2 transform between the stress pass and the Green pass (a
 * four-step DFT) and moves 30 s + 1 bytes per voxel and load instead of
 * 54 s + 1 (s = 8 in FP64, 4 in FP32); it exists for the cubic SNF grids 32,
 * 48, 64 and 96 (FP32) and 32 (FP64), with an isotropic C0 or a tabled Green
 * operator, and not for conjugate gradients.
 * The choice is dropped by lsh_set_kernel and lsh_tune_reset.  Needs the solve
 * workspace (lsh_solve_bytes); its contents are scratch.  Synchronises `stream`.
 *   out (optional): the chosen variant per pass (0 = the default), the number
 *                   of variants and each variant's mean time in ms.
 * Errors: LSH_EINVAL, LSH_ESTATE, LSH_EWORKSPACE, LSH_EDEVICE.                      */
#define LSH_TUNE_MAX 8   /* variants timed per pass, at most */
typedef struct {
  int choice[4];   /* stress pass, axis-2 passes, Green pass, schedule (0: four passes) */
  int ncand[4];
  float ms[4][LSH_TUNE_MAX];
} lsh_tune_result;

int lsh_autotune(lsh_pattern *p, int nload, lsh_precision prec, void *dev_workspace, size_t ws_bytes,
                 void *stream, lsh_tune_result *out);
int lsh_tune_reset(lsh_pattern *p);
/* Force the variants (choice[4], as in lsh_tune_result; an index beyond a
 * pass's variant count selects its last variant; a two-pass schedule where none
 * is built selects the four passes), e.g. to check each variant.                 */
int lsh_tune_set(lsh_pattern *p, lsh_precision prec, const int *choice);

/* -------------------------------------------------------------------- batches ---
 * Many microstructures and load cases in one call (the Basic Scheme of Sec. 4 for
 * each task, all advanced together).  Tasks whose patterns share M, the SNF
 * grid and the generating function form one group: each iteration is one set
 * of launches per group, and the iterations of all groups are captured in one
 * HIP graph that is replayed (two iterations per replay) on a non-default
 * stream; on the default stream the launches are issued one by one.
 *   p          : a pattern bound at prec; within a group either every C0 is
 *                isotropic (the Green operator is evaluated per instance) or all
 *                share the same C0.
 *   nload      : load cases of this task (>= 1).
 *   eps0_voigt : host nload*6 macroscopic strains; sigma_out host nload*6
 *                (nload*3 each for d = 2; tasks of 2-D and 3-D patterns may mix).
 *   stats      : optional host nload entries.
 *   dev_E_init : optional device double [nload][6][m] start fluctuation of this
 *                task (Voigt, engineering shear; [nload][3][m] for d = 2), mean
 *                removed per load as in lsh_solve; NULL = zero start.  Tasks with
 *                and without a start field may mix in one call (a warm start for
 *                some microstructures of a batch).
 *   dev_E_out  : optional device double [nload][6][m] ([nload][3][m] for d = 2)
 *                receiving this task's final E; NULL = none.
 * Both fields are double at either precision: the start field is read once per
 * solve and the output written once, against hundreds of iterations on the
 * state, so the boundary keeps the widest type and the FP32 path converts on
 * the device.  Both must stay alive until lsh_solve_batch returns.               */
typedef struct {
  lsh_pattern *p;
  int nload;
  const double *eps0_voigt;
  double *sigma_out;
  lsh_stats *stats;
  const double *dev_E_init;
  double *dev_E_out;
} lsh_task;

/* Workspace bytes for lsh_solve_batch over these tasks.                            */
int lsh_batch_bytes(const lsh_task *tasks, int ntask, lsh_precision prec, size_t *bytes);

/* Solve every task; same tolerance semantics and statuses as lsh_solve.
 * Synchronises `stream` before returning.                                          */
int lsh_solve_batch(const lsh_task *tasks, int ntask, double tol, int max_iter, lsh_precision prec,
                    void *dev_workspace, size_t ws_bytes, void *stream);

/* --------------------------------------------------------------- diagnostics ---
 * Per-kernel GPU time, from HIP event pairs recorded on the solve stream around
 * every launch and read back at the solver's own synchronisation points.
 * Slots: 0 axis-1 stress pass, 1 axis-2 forward, 2 Green pass (axis 3),
 * 3 residual reduction, 4 axis-2 inverse, 5 final effective-stress pass.
 * lsh_profile_enable(1) clears the counters and times every slot; process-wide,
 * not thread-safe.  lsh_profile_select(mask) then limits the timing to the slots
 * whose bit is set (bit i = slot i): each timed launch adds two event records to
 * the stream, and with them a few microseconds of idle time between kernels.
 * lsh_profile_read copies the first n slots (n <= 8) of the accumulated
 * milliseconds and launch counts.                                              */
int lsh_profile_enable(int on);
int lsh_profile_select(unsigned mask);
int lsh_profile_read(double *ms, long long *counts, int n);

/* Thread-local message for the last non-zero status returned on this thread.      */
const char *lsh_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* LSH_H */
