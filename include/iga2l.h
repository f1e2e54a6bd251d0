/*
 * iga2l.h -- C ABI of the MI355X (gfx950) two-level solver for B-spline
 * isogeometric discretisations of -div(kappa grad u) = f on (0,1)^d with
 * homogeneous Dirichlet conditions, after "A two level method for
 * isogeometric discretizations" (arXiv:2009.01499).
 *
 * One two-level cycle (Algorithm 1 of the paper) is: one sweep of the
 * overlapping multiplicative Schwarz smoother with p-dependent square blocks
 * (Section 3.1.1), the fine defect, restriction to the degree-1 space on the
 * same knots by the lumped L2 projection (Section 3.1.2), a coarse solve
 * (exact, or one h-multigrid V-cycle with red-black Gauss-Seidel, Section
 * 3.2), and prolongation by the adjoint of the restriction.
 *
 * Conventions shared by every entry point
 *   - Return value: IGA2L_OK (0) or a negative IGA2L_E* code; the message of
 *     the last failure on the calling thread is iga2l_last_error().  No C++
 *     exception crosses this interface.
 *   - DOF order: interior tensor-product B-splines, lexicographic with x
 *     fastest; n_fine = (m+p-2)^d, n_coarse = (m-1)^d, n_elem = m^d.
 *   - Vectors u, b, r, lambda, grad_* and the coarse vectors are caller-owned
 *     DEVICE pointers to contiguous IEEE double arrays on the problem's
 *     device.  Host arrays (knots, kappa) are copied during the call.
 *   - stream is a hipStream_t (NULL = the default stream).  All work of a
 *     call is enqueued on that stream; calls return without synchronising
 *     except iga2l_solve*, which read back the convergence record.
 *   - The problem object owns every workspace; it is not safe to run two
 *     calls on one problem concurrently.
 */
#ifndef IGA2L_H
#define IGA2L_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct iga2l_problem iga2l_problem;

enum {
    IGA2L_OK = 0,
    IGA2L_EINVAL = -1,        /* bad argument (knots, degree, kappa, pointer, option) */
    IGA2L_ENOMEM = -2,        /* device or host allocation failed */
    IGA2L_EDEVICE = -3,       /* HIP runtime error */
    IGA2L_ENOTCONV = -4,      /* max_cycles reached before tol; u holds the last iterate */
    IGA2L_ENUMERIC = -5,      /* non-positive pivot in a block, NaN/Inf residual or divergence */
    IGA2L_EUNSUPPORTED = -6   /* valid request outside what this build implements */
};

enum { IGA2L_LEX = 0, IGA2L_COLOUR = 1 };                 /* Schwarz block ordering */
enum { IGA2L_COARSE_DIRECT = 0, IGA2L_COARSE_VCYCLE = 1 };
enum { IGA2L_FP64 = 0, IGA2L_MIXED_FP32 = 1 };

typedef struct {
    double tol;          /* stop when ||b - A u||_2 <= tol * ||b - A u0||_2 (paper: 1e-8) */
    int max_cycles;      /* upper bound on two-level cycles */
    int ordering;        /* IGA2L_LEX (one block at a time, lexicographic) or IGA2L_COLOUR */
    int colour_period;   /* COLOUR only: period s >= block width; 0 selects s = block width */
    int coarse;          /* IGA2L_COARSE_DIRECT or IGA2L_COARSE_VCYCLE.  DIRECT solves the coarse
                            space exactly: kappa = 1 by the DST-I (fast diagonalisation for
                            plow = 2); variable kappa (plow = 1, at most 4096 coarse unknowns,
                            else EUNSUPPORTED at set-up) by a banded Cholesky factorisation of
                            A_1 at set-up, whose inverse the solve applies */
    int nu1, nu2;        /* pre-/post-smoothing steps of the coarse V-cycle (paper: 1, 1) */
    int precision;       /* IGA2L_FP64, or IGA2L_MIXED_FP32: FP64 residual and accumulation,
                            FP32 smoother, defect, transfers and V-cycle */
    int fine_post_sweeps;/* Schwarz sweeps after the coarse correction (paper: 0) */
    int lumped;          /* 1: restriction D^{-1} M_p^1 with the row-sum lumped degree-1 mass
                            matrix D (Section 3.1.2, the paper's choice); 0: the exact
                            L2 projection (M_1^1)^{-1} M_p^1 (M_1^1 applied through its DST-I).
                            Applies to iga2l_solve*; iga2l_restrict / iga2l_prolong follow the
                            value of the last iga2l_setup_blocks */
    int aggressive;      /* 1: aggressive coarsening (Section 3.3): the coarse level is the
                            degree-1 discretisation on the grid of size 2h, reached by the degree
                            transfer followed by linear interpolation's transpose; coarse =
                            COARSE_VCYCLE runs one V(nu1,nu2) cycle from the 2h level, COARSE_DIRECT
                            solves the 2h level exactly (kappa = 1, m even).  Needs more than 512
                            unknowns on the degree-1 level.  0: degree 1 on the same grid */
    int plow;            /* degree of the coarse space on the same knots (Section 3.1): 1 (default) or
                            2 (Section 5, for geometries that need it); 2 is solved exactly
                            (COARSE_DIRECT, kappa = 1, by fast diagonalisation of the 1-D degree-2
                            stiffness and mass matrices), with lumped or exact transfers.  Fixed by
                            iga2l_setup_blocks (which re-sizes the coarse space); n_coarse =
                            (m + plow - 2)^d */
} iga2l_opts;

typedef struct {
    int iters;                 /* cycles performed */
    int status;                /* IGA2L_OK, IGA2L_ENOTCONV or IGA2L_ENUMERIC */
    double r0;                 /* ||b - A u0||_2 */
    double relres;             /* final ||b - A u||_2 / r0 */
    double t_solve_ms;         /* wall time of the call (host clock, after the final sync) */
    double t_setup_ms;         /* wall time of iga2l_assemble and every iga2l_setup_blocks of the problem */
    double *relres_history;    /* optional host array, filled with relres after each cycle */
    int history_cap;           /* its length (0 if none) */
} iga2l_info;

/* Fill o with the defaults: tol 1e-10, 100 cycles, COLOUR with s = block
 * width, V(1,1) coarse cycle, FP64, no post-smoothing, lumped transfers,
 * degree-1 coarse level on the same grid (plow = 1). */
void iga2l_default_opts(iga2l_opts *o);

/*
 * Assemble the Galerkin system of Section 2 (stiffness a(u,v) = integral of
 * kappa grad u . grad v over the B-spline space of degree p with maximal
 * smoothness, eq. splinespace / splinespace2) and the transfer and coarse
 * operators of Section 3 (degree 1 on the same knots).
 *   dim     2 or 3 (tensor-product space; the paper treats d = 2)
 *   knots   dim host arrays: the open uniform knot vector of Section 2.1 in
 *           each direction, p+1 zeros, the interior knots i/m, p+1 ones;
 *           all directions identical.  Length nknots[k] = 2p+m+1.
 *   p       degree, 1..8 (dim 3: 1..4)
 *   kappa   host array of m^dim per-element coefficients (x fastest), each
 *           finite and > 0; NULL means kappa = 1 (the Poisson problem).
 *   device  HIP device ordinal.
 * Errors: EINVAL (knots not open/uniform, m < 2, p or dim out of range,
 * kappa <= 0 or not finite, NULL out), ENOMEM, EDEVICE.
 */
int iga2l_assemble(int dim, const double *const *knots, const int *nknots, int p,
                   const double *kappa, int device, iga2l_problem **out);

/*
 * The quarter-annulus problem of Section 5.2: -Laplace u = f on
 * {r_in^2 <= x^2 + y^2 <= r_out^2, x, y >= 0}, u = 0 on the boundary,
 * discretised with the NURBS space of Section 2.2 (eq. for R_ij^p): the
 * exact quadratic-NURBS geometry (the quarter circle as the rational
 * quadratic with weights 1, sqrt(2)/2, 1 along the angular parameter, linear
 * along the radial one) raised to degree p with maximal smoothness on m x m
 * elements, the Dirichlet functions removed (n_fine = (m+p-2)^2, x index =
 * angular parameter, fastest).  The coarse level is the degree-2 NURBS space
 * on the same elements (Section 5.2: p_low = 2), reached by the lumped L2
 * transfers of Section 3.1.2; setup_blocks / solve then need opts->plow = 2,
 * lumped = 1, coarse = COARSE_DIRECT (solved exactly, by fast
 * diagonalisation of the tensor-sum coarse operator) and no aggressive
 * coarsening.  The Schwarz blocks invert each block of the assembled operator
 * (no shared interior inverse).  Integrals use p+3 Gauss points per element
 * and direction.  solve_backward works without its grad_kappa output.
 *   p       fine degree, 2..8;  m  elements per direction, >= 2;
 *   r_in, r_out  radii, 0 < r_in < r_out (the paper: 0.3, 0.5);
 *   device  HIP device ordinal.
 * Errors: EINVAL (m < 2, radii, NULL out), EUNSUPPORTED (p), ENOMEM, EDEVICE.
 */
int iga2l_assemble_annulus(int p, int m, double r_in, double r_out, int device, iga2l_problem **out);

/*
 * Build the Schwarz blocks of Section 3.1.1 (one block per DOF: the DOFs
 * within (block_width-1)/2 of it in every direction, truncated at the
 * boundary) and invert every block matrix A^{B_j} = V_j A V_j^T on the device,
 * plus what opts asks for: FP32 copies (MIXED_FP32), the coarse V-cycle
 * hierarchy or the exact coarse solver.
 *   block_width  odd, 1..7; 0 selects the paper's choice (3 for p <= 4,
 *                5 for p = 5, 6, 7 for p = 7, 8; Sections 4.2 and 5.1).
 * May be called again to change options.  Errors: EINVAL, ENUMERIC (a block
 * matrix not positive definite), ENOMEM, EDEVICE, EUNSUPPORTED.
 */
int iga2l_setup_blocks(iga2l_problem *prob, int block_width, const iga2l_opts *opts);

/* Sizes: fine DOFs, coarse (degree-1) DOFs, elements.  Any pointer may be NULL. */
int iga2l_sizes(const iga2l_problem *prob, int64_t *n_fine, int64_t *n_coarse, int64_t *n_elem);

/* r = b - A u in FP64 (Algorithm 1, defect).  u, b, r: device, n_fine. r may not alias u. */
int iga2l_residual(const iga2l_problem *prob, const double *u, const double *b, double *r, void *stream);

/*
 * nsweeps sweeps of the multiplicative Schwarz smoother on A u = b, in place
 * on u, FP64, with opts->ordering / colour_period (COLOUR: the blocks of one
 * colour are updated together from the iterate at the start of the colour).
 * Requires iga2l_setup_blocks.  opts may be NULL (defaults).
 */
int iga2l_smooth(const iga2l_problem *prob, double *u, const double *b, int nsweeps,
                 const iga2l_opts *opts, void *stream);

/*
 * Allocation-free variant of iga2l_smooth, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc).  Same arguments and the same result, bit for bit,
 * as iga2l_smooth with the coloured ordering (opts->ordering must be
 * IGA2L_COLOUR, else EUNSUPPORTED).  The intermediate iterates of a sweep live
 * in a fixed device array of the library (2 * IGA2L_NOALLOC_MAX_FINE doubles,
 * 32 MiB, one copy per device, held until the process ends) instead of the
 * problem's workspaces; the call performs no hipMalloc, hipFree or other
 * allocation.  n_fine above IGA2L_NOALLOC_MAX_FINE: EINVAL.  Every call on
 * one device shares that array: calls that overlap on one device (other
 * streams, other threads) race and must be serialised by the caller.
 */
#define IGA2L_NOALLOC_MAX_FINE 2097152
int iga2l_smooth_noalloc(const iga2l_problem *prob, double *u, const double *b, int nsweeps,
                         const iga2l_opts *opts, void *stream);

/*
 * Measurement helper for benchmarks: the average duration in milliseconds of
 * one launch of the coloured Schwarz kernel (one colour of the sweep of
 * Section 3.1.1, colour period from opts, default the block width) in the
 * given arithmetic (IGA2L_FP64, or IGA2L_MIXED_FP32 for the FP32 kernel of
 * the mixed-precision correction cycle), timed with HIP events on stream over
 * nsweeps (>= 1) back-to-back sweeps after one warm-up sweep.  The sweeps run
 * on the problem's own correction workspaces with a zero iterate and
 * right-hand side (their previous contents are lost).  Synchronises.
 */
int iga2l_time_colour(const iga2l_problem *prob, int precision, int nsweeps, const iga2l_opts *opts,
                      void *stream, double *ms_per_launch);

/* d_coarse = D^{-1} M_p^{1} r_fine: the restriction of Section 3.1.2 with the
 * row-sum lumped degree-1 mass matrix D (with lumped = 0 at the last set-up:
 * (M_1^1)^{-1} M_p^1 r_fine).  FP64, n_fine -> n_coarse. */
int iga2l_restrict(const iga2l_problem *prob, const double *r_fine, double *d_coarse, void *stream);

/* u_fine += (M_p^{1})^T D^{-1} e_coarse: the prolongation, adjoint of the restriction. */
int iga2l_prolong(const iga2l_problem *prob, const double *e_coarse, double *u_fine, void *stream);

/* e_coarse = approximation of A_1^{-1} d_coarse by opts->coarse (exact for
 * COARSE_DIRECT; one V(nu1,nu2) cycle from zero for COARSE_VCYCLE), FP64.
 * With opts->aggressive: e_coarse = P_0 C P_0^T d_coarse, P_0 the linear
 * interpolation from the 2h grid, C the exact 2h solve or the V-cycle from
 * the 2h level (Section 3.3). */
int iga2l_coarse_solve(const iga2l_problem *prob, const double *d_coarse, double *e_coarse,
                       const iga2l_opts *opts, void *stream);

/*
 * Solve A u = b by two-level cycles from the initial guess in u until the
 * relative residual reaches opts->tol or opts->max_cycles cycles ran.
 * Returns OK, ENOTCONV (u = last iterate) or ENUMERIC; info (may be NULL)
 * receives the record.  Synchronises the stream before returning.
 */
int iga2l_solve(const iga2l_problem *prob, const double *b, double *u, const iga2l_opts *opts,
                iga2l_info *info, void *stream);

/*
 * Solve nprob independent problems (each assembled and set up with the same
 * opts) b[k] -> u[k].  infos: array of nprob records (may be NULL).
 */
int iga2l_solve_batch(iga2l_problem *const *probs, int nprob, const double *const *b,
                      double *const *u, const iga2l_opts *opts, iga2l_info *infos, void *stream);

/*
 * Adjoint of the solve, for a loss L(u) with u = A(kappa)^{-1} b:
 * lambda = A^{-1} grad_u (A is symmetric, so the same two-level solver is
 * used) and grad_kappa[e] = -integral over element e of grad(lambda_h) .
 * grad(u_h) = dL/dkappa_e.  u: the forward solution (device, n_fine);
 * grad_u (n_fine), lambda (out, n_fine), grad_kappa (out, n_elem): device.
 */
int iga2l_solve_backward(const iga2l_problem *prob, const double *u, const double *grad_u,
                         double *lambda, double *grad_kappa, const iga2l_opts *opts,
                         iga2l_info *info, void *stream);

/* Release every device and host resource of the problem (NULL is ignored). */
void iga2l_destroy(iga2l_problem *prob);

/* Message of the last non-OK return on the calling thread ("" if none). */
const char *iga2l_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* IGA2L_H */
