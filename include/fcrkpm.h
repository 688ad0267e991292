/*
 * fcrkpm.h -- C ABI of the MI355X (gfx950) FC-RKPM Poisson library.
 *
 * The library evaluates the fast-convolving reproducing kernel particle method
 * of arXiv 2403.19854 for the Galerkin Poisson problem (Sec 2.2, Eq 8-9) on a
 * uniform periodic box grid that embeds the domain (Sec 4.1, Sec 5.1): every
 * RK sum is a circular convolution computed with a hand-written 3D FFT on the
 * GPU (Sec 3, Eq 34).
 *
 * Conventions shared by every call
 *   - Arrays are DEVICE pointers owned by the caller; the library never frees
 *     or retains them past the call (setup copies what it keeps).
 *   - Node layout is C order [nz][ny][nx], x fastest; unused axes have n = 1.
 *   - Every call enqueues its work on the caller's HIP stream `stream`
 *     (NULL = the null stream).  fcrkpm_apply is asynchronous; setup, solve
 *     and adjoint synchronise the stream before returning.
 *   - A context is used from one stream at a time and is not thread-safe.
 *   - No C++ exception crosses this boundary: every call returns a status;
 *     fcrkpm_last_error(ctx) gives a message for the last failing call.
 */
#ifndef FCRKPM_H
#define FCRKPM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct fcrkpm_ctx fcrkpm_ctx;

typedef enum {
    FCRKPM_OK = 0,
    FCRKPM_ERR_ARG = 1,         /* invalid argument or geometry             */
    FCRKPM_ERR_SINGULAR = 2,    /* a moment matrix is not positive definite */
    FCRKPM_ERR_NOCONV = 3,      /* solver hit maxit or broke down           */
    FCRKPM_ERR_HIP = 4,         /* a HIP runtime call failed                */
    FCRKPM_ERR_OOM = 5,         /* device allocation failed                 */
    FCRKPM_ERR_UNSUPPORTED = 6  /* valid request not implemented            */
} fcrkpm_status;

/* Kernel functions (Sec 2.1). */
enum { FCRKPM_KERNEL_CUBIC_BSPLINE = 0 }; /* Eq 6-7: tensor-product cubic B-spline */

/* Operators of fcrkpm_apply. */
enum {
    FCRKPM_OP_K = 0,      /* chi_Omega o K (chi_Omega o d): the CG operator  (Eq 91, Alg 2, masks Eq 96) */
    FCRKPM_OP_K_FULL = 1, /* f^int = K d over all domain nodes               (Eq 57, 91; Alg 2)          */
    FCRKPM_OP_FR = 2,     /* f^r = N^T (V o r)                               (Eq 60, 92; Alg 4)          */
    FCRKPM_OP_UH = 3,     /* u^h = N d at the nodes                          (Eq 63, 94; Alg 3)          */
    FCRKPM_OP_NT = 4,     /* N^T y  (Eq 92 without V)                                                    */
    FCRKPM_OP_VN = 5,     /* V o (N z)                                                                   */
    FCRKPM_OP_M = 6,      /* f^m = M d, consistent mass (Eq C.5, C.8, C.11; Alg C.1), domain mask
                             in and out; the first call builds its coefficients (synchronous)           */
    FCRKPM_OP_FQ = 7      /* f^q = N^T (A o q), boundary flux load (Eq 28, A.4-A.5; Alg A.1) with the
                             areas A of fcrkpm_set_boundary; FCRKPM_ERR_ARG without them                */
};

/* Number types. */
enum { FCRKPM_F64 = 0, FCRKPM_F32 = 1 };

/* Solver modes. */
enum {
    FCRKPM_MODE_F64 = 0,         /* FP64 CG on FP64 FFT products                           */
    FCRKPM_MODE_F32_REFINED = 1, /* FP32 CG inside FP64 iterative refinement (FP64 residual) */
    FCRKPM_MODE_F32_PRODUCTS = 2 /* FP64 CG vectors, FP32 K products, FP64 residual replacement */
};

/* Coefficient fields readable with fcrkpm_get_coeffs. */
enum {
    FCRKPM_COEF_B0 = 0,     /* b^0_p, p < s: first row of M^-1 (Eq 45, 83); [s][nodes]            */
    FCRKPM_COEF_BALPHA = 1, /* b^a_p: minus row a+1 of M^-1 (Eq 46-47, 84-85); [dim][s][nodes]    */
    FCRKPM_COEF_FREE = 2,   /* chi_Omega as 0/1 doubles (Eq 96); [nodes]                           */
    FCRKPM_COEF_LUMPED_MASS = 3 /* M^l, row sums of M (Eq C.9-C.10, C.13; Alg C.2); [nodes]        */
};

/* Time schemes of fcrkpm_transient (App. C.3). */
enum {
    FCRKPM_TIME_IMPLICIT = 0,        /* theta method, one CG solve per step (Alg C.4) */
    FCRKPM_TIME_EXPLICIT_LUMPED = 1  /* forward Euler with the lumped mass (Alg C.3)  */
};

typedef struct {
    int32_t scheme;  /* FCRKPM_TIME_*                                                     */
    int32_t nsteps;  /* time steps, >= 0                                                  */
    double dt;       /* step size, > 0                                                    */
    double nu;       /* diffusivity nu of Eq C.1, > 0                                     */
    double theta;    /* implicit scheme: 0 < theta <= 1 (1 backward Euler, 0.5 Crank-
                        Nicolson); ignored by the explicit scheme                         */
} fcrkpm_time;

typedef struct {
    int32_t dim;              /* spatial dimension d: 1, 2 or 3                             */
    int32_t n[3];             /* box nodes per axis (x, y, z); unused axes must be 1        */
    double h[3];              /* nodal spacing per axis (Eq 70)                             */
    const uint8_t* dirichlet; /* device: chi_Gamma_g per node (Eq 95), subset of the mask,
                                 or NULL for no Dirichlet nodes                             */
    const double* vol;        /* device: nodal volume V per node (Eq 87), or NULL for
                                 V = h_x h_y h_z on every domain node                       */
    int32_t flags;            /* reserved, must be 0                                        */
} fcrkpm_grid;

typedef struct {
    int32_t iters;          /* CG iterations (sum over inner solves in refined mode)          */
    int32_t outer_iters;    /* refinement steps (0 in FP64 mode)                              */
    double rel_res;         /* final recursive relative residual                              */
    double true_rel_res;    /* ||b - K d|| / ||b|| recomputed in FP64 at the end              */
    int32_t fallback_used;  /* 1 if refined mode fell back to FP64 CG after stagnation        */
    int32_t matvecs_f64;    /* FP64 K products issued                                         */
    int32_t matvecs_f32;    /* FP32 K products issued                                         */
} fcrkpm_info;

/*
 * fcrkpm_setup -- build a context for one box grid and domain.
 *
 * Runs the setup half of the method: kernel/basis spectra (Sec 5.2-5.3,
 * Eq 68-79), the moment convolutions M_pq = (1-chi) delta_pq + chi o
 * F^-1[F(chi) o F(H_p H_q^a)] (Sec 4.2.1, Eq 49, 80; Alg 1) and the per-node
 * moment solves giving b^0 and b^a (Eq 83-85), all in FP64.
 *
 *   grid     box geometry, Dirichlet mask and volumes (copied)
 *   mask     device: chi per node (Eq 40), 0/1 bytes (copied)
 *   kernel   FCRKPM_KERNEL_CUBIC_BSPLINE
 *   support  normalised support a~ per axis, a = a~ h (Eq 64); unused axes ignored
 *   degree   monomial degree n of the basis (Eq 4): 1 or 2, or 3 in 1D and 2D
 *   stream   HIP stream (hipStream_t) the setup runs on
 *   out      receives the new context (NULL on failure)
 *
 * Errors: FCRKPM_ERR_ARG for a bad dimension, box size (each active axis must
 * factor into 2, 3, 5, 7 and be at least 4 and at most 1024), support (1 <= a~,
 * floor(a~) < n/2), degree, a Dirichlet node outside the mask, or a mask
 * whose extent on an axis leaves a periodic gap under (floor(a~)+1) nodes
 * (Sec 5.1, Eq 66: the wrap-around would couple the two ends).  A mask that
 * occupies every index of an axis is periodic along that axis (the chi = 1
 * special case of Sec 4.2.4);
 * FCRKPM_ERR_SINGULAR if a moment matrix is not positive definite (the
 * message names the first node); FCRKPM_ERR_OOM; FCRKPM_ERR_HIP.
 */
fcrkpm_status fcrkpm_setup(const fcrkpm_grid* grid, const uint8_t* mask, int32_t kernel,
                           const double support[3], int32_t degree, void* stream,
                           fcrkpm_ctx** out);

/*
 * fcrkpm_apply -- one operator on nrhs fields, asynchronously on `stream`.
 *
 *   op      FCRKPM_OP_*
 *   dtype   FCRKPM_F64 (in/out are double*) or FCRKPM_F32 (float*): the
 *           precision of the FFT products and pointwise arithmetic
 *   nrhs    number of fields; field j starts at j * (nodes) in `in` and `out`
 *   in,out  device arrays; must not overlap
 *
 * The kernel is a tensor product (Eq 6), so every 3D spectral product of
 * Alg 2-4 is separable: instead of the paper's 3D transforms (2(s+1) per
 * field for K, s+1 for FR, UH, NT, VN) each operator runs as line passes.  In
 * 3D: part-1 passes along x and y (d -> its x-convolutions -> their
 * y-convolutions), one middle pass along z (the part-1 z-convolutions, the
 * pointwise stage and the part-2 z-convolutions, without leaving the chip),
 * then part-2 passes along y and x.  FR and NT start at the middle pass, UH
 * ends in it; 1D and 2D drop the absent axes.  The results equal the 3D
 * transforms' (circular convolutions either way).  Errors: FCRKPM_ERR_ARG
 * (bad op/dtype/nrhs, NULL or overlapping pointers), FCRKPM_ERR_HIP.
 */
fcrkpm_status fcrkpm_apply(fcrkpm_ctx* ctx, int32_t op, int32_t dtype, int32_t nrhs,
                           const void* in, void* out, void* stream);

/*
 * fcrkpm_apply_noalloc -- fcrkpm_apply for callers that cannot allocate device
 * memory (work under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc): the same operators, arguments, results and errors, but
 * the passes keep their intermediate fields in a static scratch array of
 * 64 MiB that every GPU the library runs on holds until the process ends,
 * instead of the context's workspace.  The call allocates nothing.
 *
 * Scratch need: 2 x (pair fields of the widest intermediate set) x nodes x
 * nrhs complex values, 8 bytes each in FP32 and 16 in FP64 -- for the linear
 * basis in 3D, 32 bytes (FP32) or 64 bytes (FP64) per node and right-hand
 * side: a 128^3 box fits in FP32 with one right-hand side, a 96^3 box in FP64
 * with one.  A larger request returns FCRKPM_ERR_ARG (the message gives the
 * need and the limit) before any work is enqueued.  FCRKPM_OP_M needs its
 * coefficients built by one earlier fcrkpm_apply(FCRKPM_OP_M) call
 * (FCRKPM_ERR_ARG otherwise).
 *
 * All calls on one GPU share its scratch array: calls that overlap in time on
 * one GPU (different streams, threads or contexts) race and give wrong
 * results; serialise them.  No value of the scratch survives into a result of
 * a later call (every pass writes what it reads within the call).
 */
fcrkpm_status fcrkpm_apply_noalloc(fcrkpm_ctx* ctx, int32_t op, int32_t dtype, int32_t nrhs,
                                   const void* in, void* out, void* stream);

/*
 * fcrkpm_solve -- static strong-Dirichlet solve (Sec 2.4, Eq 29; Sec 5.4.3,
 * Alg 5): d = g on Dirichlet nodes, f^r from r (Alg 4), right-hand side
 * b = chi_Omega o (f^r - K d_Gamma), CG on the free nodes (Eq 96) until
 * ||r_k||_2 / ||b||_2 <= tol on the recursive residual.
 *
 *   mode     FCRKPM_MODE_F64 or FCRKPM_MODE_F32_REFINED (FP32 inner CG,
 *            FP64 outer residual b - K d; falls back to FP64 CG if the
 *            refinement stagnates)
 *   nrhs     number of right-hand sides (fields laid out back to back); they
 *            iterate together, every pass and CG kernel covering all of
 *            them in one launch, and each stops on its own tolerance
 *   r        device FP64 source per node (Eq 8)
 *   g        device FP64 Dirichlet values per node, or NULL for g = 0
 *   d_inout  device FP64: initial guess on the free nodes in (zeros = the
 *            paper's start), solution coefficients out
 *   uh_out   device FP64 u^h = N d (Alg 3), or NULL
 *   tol      relative residual target (> 0)
 *   maxit    iteration cap (CG iterations in total, shared by the
 *            right-hand sides of the call)
 *   info     array of nrhs records, one per right-hand side (may be NULL)
 *
 * Blocks of 8 CG iterations are captured once into a HIP graph and replayed
 * (see FCRKPM_OPT_GRAPHS); the host polls convergence between blocks.
 *
 * Acceptance.  FCRKPM_MODE_F64 converges when the recursive residual reaches
 * tol.  The refined modes converge on the FP64 true residual ||b - K d|| /
 * ||b||: when it reaches tol, or when it has stopped improving (three
 * replacements in a row above half of its best) with its best within 4 tol,
 * which is then taken as the attainable accuracy (d is the best iterate).
 * A stall above 4 tol, a breakdown or divergence of the FP32 recursion hands
 * the right-hand side to FP64 CG from its best iterate.  At the end the true
 * residual is recomputed; a refined solve whose final true residual exceeds
 * 100 tol reports FCRKPM_ERR_NOCONV even if its last phase converged.
 * info.true_rel_res always holds that final value.
 *
 * Returns FCRKPM_ERR_NOCONV with the best d written when maxit is reached or
 * CG breaks down (p^T K p <= 0) for any right-hand side; FCRKPM_ERR_ARG for
 * NaN/Inf in r, g or the initial guess, or bad arguments.
 */
fcrkpm_status fcrkpm_solve(fcrkpm_ctx* ctx, int32_t mode, int32_t nrhs, const double* r,
                           const double* g, double* d_inout, double* uh_out, double tol,
                           int32_t maxit, fcrkpm_info* info, void* stream);

/*
 * fcrkpm_set_boundary -- boundary areas A of the flux nodes Gamma_q (Eq 28,
 * A.2, A.7): the quadrature weight of every boundary node that carries a flux,
 * 0 elsewhere; nodes outside the domain are ignored.
 *
 *   area    device FP64 per node (copied), or NULL to remove the areas
 *   stream  HIP stream the copy runs on (synchronised)
 *
 * Errors: FCRKPM_ERR_ARG (non-finite area), FCRKPM_ERR_OOM, FCRKPM_ERR_HIP.
 */
fcrkpm_status fcrkpm_set_boundary(fcrkpm_ctx* ctx, const double* area, void* stream);

/*
 * fcrkpm_solve_flux -- fcrkpm_solve with a flux boundary (Sec 2.2-2.4, Eq 8-9,
 * 28-29; Alg A.1): right-hand side b = chi_Omega (f^r + f^q - K d_Gamma) with
 * f^q = N^T (A o q) over the areas of fcrkpm_set_boundary.
 *
 *   q       device FP64 flux grad u . n per node (meaningful where A > 0), laid
 *           out like r; every other argument as in fcrkpm_solve
 *
 * Errors: as fcrkpm_solve; FCRKPM_ERR_ARG without boundary areas or for NaN/Inf
 * in q.
 */
fcrkpm_status fcrkpm_solve_flux(fcrkpm_ctx* ctx, int32_t mode, int32_t nrhs, const double* r,
                                const double* q, const double* g, double* d_inout, double* uh_out,
                                double tol, int32_t maxit, fcrkpm_info* info, void* stream);

/*
 * fcrkpm_nonlinear_force -- f^N = N^T (V o kappa (u^h)^3) with u^h = N d, the
 * nonlinear force of N(u) = kappa u^3 (App. B, Eq B.2, B.4, B.9; Alg B.2), FP64,
 * asynchronous on `stream`; d and out hold nrhs fields and may be the same array.
 * Errors: FCRKPM_ERR_ARG (NULL arrays, nrhs, non-finite kappa), FCRKPM_ERR_HIP.
 */
fcrkpm_status fcrkpm_nonlinear_force(fcrkpm_ctx* ctx, double kappa, int32_t nrhs, const double* d,
                                     double* out, void* stream);

/*
 * fcrkpm_gradient_force -- f^N = B^T (V o N(B d)) with the gradient
 * nonlinearity N(g) = (1 + kappa |g|^2) g (App. B, Eq B.5-B.8, B.10; Alg B.1):
 * the passes of K with N applied to the implicit gradient at every node, so
 * kappa = 0 gives K d (domain mask in and out), FP64, asynchronous on `stream`
 * (except the first call on the register path, which builds its records);
 * d and out hold nrhs fields and must not overlap.  Where the FP64 register
 * path serves the box (FCRKPM_OPT_KN_REGPATH), its middle pass applies each z
 * line's constant gradient and divergence coefficients in the spectral domain
 * with N between them and corrects the nodes near the domain's z ends directly
 * (12 transforms per line pair; kappa = 0 then equals K d to rounding).
 * Errors: FCRKPM_ERR_ARG (NULL or overlapping arrays, nrhs, non-finite kappa),
 * FCRKPM_ERR_HIP.
 */
fcrkpm_status fcrkpm_gradient_force(fcrkpm_ctx* ctx, double kappa, int32_t nrhs, const double* d,
                                    double* out, void* stream);

/*
 * fcrkpm_solve_nonlinear -- static solve of -lap u + kappa u^3 = r with d = g on
 * the Dirichlet nodes (Eq 8-9 with the term of Eq B.1; App. B.3): Newton's
 * method on R(d) = K d + f^N(d) - f^r over the free rows from d_inout, every
 * step solving (K + N^T diag(3 kappa V (u^h)^2) N) delta = -R to `tol` with the
 * solver of fcrkpm_solve (mode F64 or F32_REFINED); the Jacobian runs the K
 * passes with the rows b^a and the row b^0 weighted by sqrt(3 kappa) |u^h|.
 *
 *   kappa       coefficient of the cubic term, >= 0 (the energy stays convex)
 *   r, g        device FP64 source and Dirichlet values (g may be NULL), one field
 *   d_inout     device FP64 initial guess on the free nodes in, solution out
 *   uh_out      device FP64 u^h = N d, or NULL
 *   tol, maxit  tolerance and iteration cap of every Newton step's CG solve
 *   newton_tol  stop when ||R|| <= newton_tol ||chi_Omega f^r||
 *   maxnewton   Newton step cap (>= 1)
 *   info        one record: iters = CG iterations of all steps, outer_iters =
 *               Newton steps, rel_res = true_rel_res = final ||R|| / ||chi_Omega f^r||
 *
 * Allocates five node fields for the call and rebuilds the Jacobian's
 * coefficient rows every step (freed at the end).  Errors: FCRKPM_ERR_ARG
 * (bad mode, tol, maxit, kappa, newton_tol, maxnewton, NULL or non-finite
 * inputs); FCRKPM_ERR_NOCONV when newton_tol is not reached within maxnewton
 * steps (d holds the last iterate).
 */
fcrkpm_status fcrkpm_solve_nonlinear(fcrkpm_ctx* ctx, int32_t mode, double kappa, const double* r,
                                     const double* g, double* d_inout, double* uh_out, double tol,
                                     double newton_tol, int32_t maxnewton, int32_t maxit,
                                     fcrkpm_info* info, void* stream);

/* Nonlinear forces of fcrkpm_solve_nonlinear_cg (App. B.1). */
enum {
    FCRKPM_NONLIN_CUBIC = 0,    /* N(u) = kappa u^3 in the force N^T N(u^h)               (Eq B.2, B.4, B.9) */
    FCRKPM_NONLIN_GRADIENT = 1  /* N(grad u) = (1 + kappa |grad u|^2) grad u in B^T N    (Eq B.6, B.8, B.10) */
};

/*
 * fcrkpm_solve_nonlinear_cg -- the static nonlinear problem by nonlinear
 * conjugate gradients (App. B.3, Alg B.3): from d_inout (d = g on the
 * Dirichlet nodes), repeated force evaluations (Alg B.1/B.2) drive the
 * residual over the free rows
 *     FCRKPM_NONLIN_CUBIC:    R(d) = K d + N^T (V kappa (N d)^3) - f^r
 *     FCRKPM_NONLIN_GRADIENT: R(d) = B^T (V (1 + kappa |B d|^2) B d) - f^r
 * to ||R|| <= tol ||chi_Omega f^r||.  Both are gradients of convex energies
 * (kappa >= 0), so the minimiser is unique; directions are Polak-Ribiere with
 * restarts, steps an exact line search: the energy's derivative along the
 * direction is a cubic in the step whose coefficients one pass over the nodes
 * gives, and its root is found on the host by safeguarded Newton steps.  FP64
 * throughout (the gradient form on the FP64 register path where
 * FCRKPM_OPT_KN_REGPATH reads 1); one field.
 *
 *   kind        FCRKPM_NONLIN_*
 *   kappa       >= 0
 *   r, g        device FP64 source and Dirichlet values (g may be NULL)
 *   d_inout     device FP64 initial guess on the free nodes in (zeros = Alg
 *               B.3's start), solution out
 *   uh_out      device FP64 u^h = N d, or NULL
 *   tol, maxit  residual target and iteration cap
 *   info        one record (may be NULL): iters = nonlinear CG iterations,
 *               outer_iters = line-search Newton steps (host arithmetic on the
 *               cubic), rel_res = true_rel_res
 *               = final ||R|| / ||chi_Omega f^r||, matvecs_f64 = K-type products
 *
 * Allocates its work vectors for the call (about 10 node fields).  Errors:
 * FCRKPM_ERR_ARG (kind, kappa, tol, maxit, NULL or non-finite inputs);
 * FCRKPM_ERR_NOCONV when tol is not reached within maxit (d holds the last
 * iterate).
 */
fcrkpm_status fcrkpm_solve_nonlinear_cg(fcrkpm_ctx* ctx, int32_t kind, double kappa, const double* r,
                                        const double* g, double* d_inout, double* uh_out, double tol,
                                        int32_t maxit, fcrkpm_info* info, void* stream);

/*
 * fcrkpm_transient -- time stepping of the diffusion problem (App. C, Eq C.1-
 * C.4): M d' + nu K d = f^r with strong Dirichlet values d = g held on the
 * Dirichlet nodes and a source r constant in time.  With x the free part of d
 * and c0 = dt (f^r - nu K d_Gamma), every step solves on the free nodes
 *   FCRKPM_TIME_IMPLICIT:        (M + theta dt nu K) x1 = (M - (1-theta) dt nu K) x0 + c0
 *                                by CG from x0 (the solver of fcrkpm_solve, mode
 *                                F64 or F32_REFINED, on the shifted operator, whose
 *                                products run the K passes with the coefficient rows
 *                                sqrt(theta dt nu) b^a and b^0; Alg C.1, C.4);
 *   FCRKPM_TIME_EXPLICIT_LUMPED: x1 = x0 + (c0 - dt nu K x0) / M^l   (Alg C.2, C.3;
 *                                FP64 products; stable for dt nu lambda_max < 2).
 *
 *   tp       scheme, nsteps, dt, nu, theta (fcrkpm_time)
 *   mode     FCRKPM_MODE_F64 or FCRKPM_MODE_F32_REFINED (implicit); F64 (explicit)
 *   nrhs     fields stepped together, laid out back to back
 *   r        device FP64 source per node, or NULL for r = 0
 *   g        device FP64 Dirichlet values per node, or NULL for g = 0
 *   d_inout  device FP64 coefficients at t = 0 in (values on the Dirichlet nodes
 *            are replaced by g), coefficients at t = nsteps dt out
 *   uh_out   device FP64 u^h = N d at the final time (Alg 3), or NULL
 *   tol      relative residual target of every step's solve (> 0)
 *   maxit    CG iteration cap of every step's solve
 *   info     nrhs records (may be NULL): iterations and products summed over
 *            the steps, the largest residuals of any step
 *
 * Allocates a work field of nrhs x nodes doubles for the call; the coefficient
 * rows of M and of the shifted operator stay with the context (the latter is
 * rebuilt when theta dt nu changes).  Errors: FCRKPM_ERR_ARG (bad scheme,
 * dt, nu, theta, nsteps, tol, maxit, NULL pointers, non-finite inputs);
 * FCRKPM_ERR_UNSUPPORTED (explicit scheme in another mode);
 * FCRKPM_ERR_SINGULAR (a lumped mass entry <= 0 on a free node);
 * FCRKPM_ERR_NOCONV (a step's solve missed tol: stepping stops there and d
 * holds that step's best iterate).
 */
fcrkpm_status fcrkpm_transient(fcrkpm_ctx* ctx, const fcrkpm_time* tp, int32_t mode, int32_t nrhs,
                               const double* r, const double* g, double* d_inout, double* uh_out,
                               double tol, int32_t maxit, fcrkpm_info* info, void* stream);

/*
 * fcrkpm_solve_batch -- fcrkpm_solve for a ragged batch of problems: nprob
 * contexts (distinct; box sizes may differ), problem p with nrhs[p]
 * right-hand sides r[p], Dirichlet values g[p] (g or g[p] may be NULL),
 * d_inout[p] and uh_out[p] (uh_out or uh_out[p] may be NULL), as in
 * fcrkpm_solve.  All problems iterate together on `stream`: each block of 8
 * CG iterations of every unfinished problem is one captured HIP graph whose
 * per-problem branches run concurrently, re-captured only when a problem
 * finishes or changes phase.  info, if not NULL, holds sum(nrhs) records,
 * problem by problem.  Status: the worst of the problems; the message is set
 * on every context of the batch.
 */
fcrkpm_status fcrkpm_solve_batch(fcrkpm_ctx* const* ctxs, int32_t nprob, int32_t mode,
                                 const int32_t* nrhs, const double* const* r,
                                 const double* const* g, double* const* d_inout,
                                 double* const* uh_out, double tol, int32_t maxit,
                                 fcrkpm_info* info, void* stream);

/*
 * fcrkpm_adjoint -- gradient of a loss of u^h(r) with respect to the source.
 *
 * With u^h = N d(r) and d(r) the homogeneous solution of fcrkpm_solve,
 * f^r = N^T V r (Eq 59) and u^h = N d (Eq 62) give
 *     dL/dr = V o N z,   z = K_ff^-1 chi_Omega o N^T (dL/du^h),
 * K being symmetric (Eq 26).
 *
 *   dl_duh   device FP64 dL/du^h per node
 *   dl_dr    device FP64 result per node
 * Other arguments and errors as fcrkpm_solve.
 */
fcrkpm_status fcrkpm_adjoint(fcrkpm_ctx* ctx, int32_t mode, int32_t nrhs, const double* dl_duh,
                             double* dl_dr, double tol, int32_t maxit, fcrkpm_info* info,
                             void* stream);

/*
 * fcrkpm_get_coeffs -- copy a coefficient field into a caller buffer
 * (device FP64), e.g. for checking the moment solves.  `which` is
 * FCRKPM_COEF_*; sizes are given with the enum.  Asynchronous on `stream`.
 */
fcrkpm_status fcrkpm_get_coeffs(fcrkpm_ctx* ctx, int32_t which, double* out, void* stream);

/*
 * Measurement hooks (not part of the method).  fcrkpm_profile(ctx, 1) opens a
 * sampling window: for every kernel kind the library launches, HIP events on
 * the launch stream bracket the first 64 launches, and every launch is counted
 * with its algorithmic bytes (the bytes the launch must read and write, from
 * the array sizes).  fcrkpm_profile(ctx, 0) closes the window and keeps the
 * samples.  fcrkpm_profile_read synchronises the device and returns, for one
 * kind, the launches counted, the mean duration of the sampled launches in ms
 * and the mean algorithmic bytes per launch.  Kinds are 0 ..
 * fcrkpm_kernel_kinds()-1; fcrkpm_kernel_name names them ("" if out of range).
 */
fcrkpm_status fcrkpm_profile(fcrkpm_ctx* ctx, int32_t enable);
fcrkpm_status fcrkpm_profile_read(fcrkpm_ctx* ctx, int32_t kind, int64_t* launches,
                                  double* mean_ms, double* bytes_per_launch);
int32_t fcrkpm_kernel_kinds(void);
const char* fcrkpm_kernel_name(int32_t kind);

/* Options of a context, set with fcrkpm_set_option. */
enum {
    FCRKPM_OPT_GRAPHS = 1,  /* 1 (default): CG blocks replay captured HIP graphs; 0: direct
                               launches.  Graphs are never used while profiling is on. */
    FCRKPM_OPT_REGPATH = 2,  /* 1 (default): K-type products on 3D boxes whose axes are
                                register-path lengths use register-resident line transforms:
                                FP32 (K, the consistent mass and the shifted and Jacobian
                                operators built from them) at 32, 48, 64, 80, 96, 128 and 256
                                points with the linear basis and at 64 and 128 with the
                                quadratic basis (K only); FP64 (K, the consistent mass, the
                                gradient force, the implicit gradient, u^h and f^r) at 32, 48,
                                64, 80, 96, 128 and 256 points with the linear basis and the
                                line-constant middle pass; 0: the LDS-tiled passes used
                                everywhere else */
    FCRKPM_OPT_REGLAYOUT = 3, /* variant of those transforms, layout + 2 (tiles - 1): layout 0 =
                                 8 lanes per line, 1 = 16 lanes (128-point lines only); at 80
                                 and 96 points layout 0 = 16 lanes x 8 values (a DFT-5 or
                                 DFT-6 first stage), 1 = 8 lanes; at 256 points
                                 layout 0 = 16 lanes x 16 points, 1 = 32 lanes x 8 points;
                                 tiles = 1 or 2 tiles per workgroup (64 and 128 points; the
                                 second tile's loads overlap the first tile's work).  Setup
                                 times a K product with each variant and keeps the fastest.
                                 FP64 products use the 16-lane layout at 80 and 96 points and
                                 the 32-lane one at 256. */
    FCRKPM_OPT_TUNE_NS0 = 4, /* read only: setup's time of one K product with variant 0, ns */
    FCRKPM_OPT_TUNE_NS1 = 5, /* read only: the same with variant 1 (0 where not timed) */
    FCRKPM_OPT_TUNE_NS2 = 6, /* read only: the same with variant 2 */
    FCRKPM_OPT_TUNE_NS3 = 7, /* read only: the same with variant 3 */
    FCRKPM_OPT_LINECONST = 8, /* 1 (default): where every z line of the box has a constant
                                pointwise matrix V B^T B away from the few nodes near the ends
                                of the domain's z extent (cube-like domains, linear basis, K),
                                the register path's middle pass applies that constant in the
                                spectral domain and corrects the end nodes directly (the same
                                sums as Alg 2, regrouped); 0: the middle pass with a pointwise
                                stage at every node.  Reads 1 only where setup found the
                                structure. */
    FCRKPM_OPT_SEP_LINES32 = 9,  /* LDS-tiled passes, FP32: most lines per workgroup (16, 8, 4) */
    FCRKPM_OPT_SEP_LINES64 = 10, /* the same for FP64.  Setup times K products with each on the
                                    precisions that run on these passes and keeps the fastest. */
    FCRKPM_OPT_TUNE_CACHED = 11, /* read only: 1 if setup took its tuning choices from the file
                                    named by FCRKPM_AUTOTUNE_CACHE (keyed by device, box, basis
                                    and support) instead of timing; new choices are appended to
                                    that file */
    FCRKPM_OPT_KN_REGPATH = 12   /* read only: 1 if fcrkpm_gradient_force (and the gradients of
                                    fcrkpm_solve_nonlinear_cg) run on the FP64 register path;
                                    the first read builds that path's records (synchronous) */
};
/* Set an option; FCRKPM_ERR_ARG for an unknown option or a value out of range. */
fcrkpm_status fcrkpm_set_option(fcrkpm_ctx* ctx, int32_t option, int64_t value);
/* Read an option into *value. */
fcrkpm_status fcrkpm_get_option(fcrkpm_ctx* ctx, int32_t option, int64_t* value);

/* Basis size s = (n+d)!/(d! n!) of the context (Eq 5), or -1 for NULL. */
int32_t fcrkpm_basis_size(const fcrkpm_ctx* ctx);

/* Release a context; NULL is a no-op. */
void fcrkpm_destroy(fcrkpm_ctx* ctx);

/* Message of the last failing call on ctx ("" if none); ctx may be NULL for
 * failures of fcrkpm_setup before a context existed. */
const char* fcrkpm_last_error(const fcrkpm_ctx* ctx);

/* Static name of a status code. */
const char* fcrkpm_status_str(fcrkpm_status s);

/* Library version, major * 10000 + minor * 100 + patch. */
int32_t fcrkpm_version(void);

#ifdef __cplusplus
}
#endif

#endif /* FCRKPM_H */
