/*
 * iss.h -- C ABI of the MI355X (gfx950) matrix-free Stokes hot path.
 *
 * Method: Huber, Ruede, Waluga, Wohlmuth, "Highly sparse surface couplings
 * for subdomain-wise isoviscous Stokes finite element discretizations"
 * (arXiv:1604.07994).  Stabilised P1-P1 Stokes on uniformly refined
 * simplicial macro meshes (Kuhn lattices), piecewise constant viscosity,
 * and on the whole boundary either homogeneous Dirichlet velocity (no-slip,
 * the default) or free-slip, u . n = 0 with zero tangential traction
 * (eq. boundary; option bc).  The viscous block
 * is one of
 *   ISS_GRADIENT   (mu grad u, grad v) everywhere (Sec. 1; inconsistent),
 *   ISS_STRAIN     a_sym = (2 mu sym grad u, sym grad v)   (eq. standard),
 *   ISS_INTERFACE  a_tr = a_sym - (mu div u, div v)        (eq. newbil),
 *                  applied as in eq. equivalence-stencil: the decoupled
 *                  Laplacian stencil per component on isoviscous rows and
 *                  the full a_tr rows only at interface vertices and, for
 *                  free-slip, at boundary vertices (Gamma_F, Sec. 2.2).
 * The saddle-point matrix is K = [[A, B^T], [B, -C]] (Sec. 5) with the
 * weak divergence b(v, q) = -(div v, q) (eq. weaks) and the pressure
 * stabilisation c(p, q) = sum_T beta h^2 / mu_T (grad p, grad q)_T.
 *
 * Vector layout (every vector argument).  A level with n cells per axis has
 * N = (n+1)^d lattice vertices, vertex v = i + (n+1) (j + (n+1) k), x
 * fastest, coordinates (i, j, k) / n on the unit cube (square).  A vector
 * is d+1 contiguous fields [u_1 | ... | u_d | p], each of length N, so
 * (d+1) N elements in total.  Fixed velocity entries -- every component of
 * a boundary vertex for no-slip; for free-slip component k of a vertex on
 * a face x_k = 0 or 1 -- are zero Dirichlet values: inputs must hold 0
 * there and outputs hold 0 there.
 * Pressure lives on every vertex.  Element type: double for ISS_FP64,
 * float for ISS_FP32, bfloat16 (1-8-7 bits, round to nearest even) for
 * ISS_FP32_BF16STORE and IEEE half (1-5-10 bits) for ISS_FP32_FP16STORE,
 * both with FP32 arithmetic (see each call).
 *
 * Memory ownership.  Vector arguments are device pointers owned by the
 * caller (any allocator; 8-byte aligned).  The library allocates and owns
 * its metadata (hipMalloc at create time) and the coarse factorisation or
 * the coarse Krylov vectors (at their first use).
 * Its work vectors (per-level V-cycle and smoother buffers, the FGMRES
 * basis) come from a workspace the caller binds with iss_bind_workspace,
 * or, if none is bound, from hipMalloc at their first use; iss_problem_
 * destroy frees what the library allocated.
 *
 * Streams.  Every call enqueues its kernels on the given stream and returns
 * without synchronising, except calls that return host scalars
 * (iss_residual with norms, iss_dot, iss_solve), which synchronise that
 * stream before returning.
 *
 * Errors.  Every int-returning call returns ISS_OK (0) or a negative code;
 * iss_last_error() gives a message for the calling thread.  No C++
 * exception crosses the ABI.
 */
#ifndef ISS_H
#define ISS_H

#include <stdint.h>
#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ihipStream_t* iss_stream_t; /* same type as hipStream_t */

typedef struct iss_problem iss_problem;   /* opaque, library owned */

enum iss_status {
    ISS_OK = 0,
    ISS_E_INVAL = -1,     /* bad argument (form, level, size, pointer)      */
    ISS_E_HIP = -2,       /* a HIP runtime call failed                      */
    ISS_E_NOTCONV = -3,   /* maxit reached before the tolerance; info set   */
    ISS_E_DIVERGED = -4,  /* residual grew by more than 1e3 or is NaN/Inf   */
    ISS_E_NOMEM = -5,     /* device or host allocation failed               */
    ISS_E_NOWS = -6       /* the bound workspace is too small               */
};

enum iss_form { ISS_GRADIENT = 0, ISS_STRAIN = 1, ISS_INTERFACE = 2 };
enum iss_block { ISS_VELOCITY_ONLY = 0, ISS_FULL_STOKES = 1 };
enum iss_prec { ISS_FP64 = 0, ISS_FP32 = 1, ISS_FP32_BF16STORE = 2, ISS_FP32_FP16STORE = 3 };
enum iss_outer { ISS_OUTER_RICHARDSON = 0, ISS_OUTER_FGMRES = 1 };
enum iss_inclusion_kind { ISS_SPHERE = 0, ISS_HALFSPACE = 1, ISS_BOX = 2 };
enum iss_bc { ISS_BC_NOSLIP = 0, ISS_BC_FREESLIP = 1 };
enum iss_coarse_solver { ISS_COARSE_DIRECT = 0, ISS_COARSE_MINRES = 1 };
enum iss_coarse_mu { ISS_COARSE_MU_CENTROID = 0, ISS_COARSE_MU_AVERAGE = 1 };

/* A viscosity inclusion.  Sphere: a = (cx, cy, cz, r, -, -), region
 * |x-c| < r (cz ignored in 2D).  Half-space: a = (axis, threshold, -, ..),
 * region x[axis] < threshold.  Box: a = (x0, x1, y0, y1, z0, z1), region
 * x0 < x < x1, y0 < y < y1, z0 < z < z1 (z ignored in 2D; the viscosity
 * columns of Sec. 4 are two such boxes).  An element takes the phase of
 * the first inclusion
 * (array order) whose region contains its centroid, else phase 0 (the
 * unresolved-interface setting of the remark closing Sec. 2.2). */
typedef struct {
    int kind;
    int phase;            /* 1..nphase-1 */
    double a[6];
} iss_inclusion;

typedef struct {
    int nu1, nu2;         /* pre/post Uzawa smoothing steps (3, 3; Sec. 5)  */
    double omega;         /* pressure under-relaxation (0.3; Sec. 5)        */
    double stab_beta;     /* stabilisation constant beta (1/12)             */
    int outer;            /* ISS_OUTER_RICHARDSON or ISS_OUTER_FGMRES       */
    int restart;          /* FGMRES restart length (default 40)             */
    int coarse_mu;        /* viscosity of coarse-level elements:
                           * ISS_COARSE_MU_CENTROID: centroid rule on each
                           *   level (plain rediscretisation);
                           * ISS_COARSE_MU_AVERAGE (default): volume average
                           *   of the nested finest-level viscosities (and of
                           *   1/mu for C) -- for nested P1 spaces the coarse
                           *   viscous block is then the Galerkin product
                           *   P^T A P.  A level keeps its distinct
                           *   averages exactly when they fit its 254-entry
                           *   phase table; otherwise the mixed averages are
                           *   grouped into <= 250 logarithmic bins (each
                           *   member takes its bin's mean; relative width
                           *   below 4% at contrast 1e4), an approximation
                           *   of the preconditioner only.                 */
    int coarse_form;      /* viscous form of the coarsest level inside
                           * V-cycles (Sec. 5 swaps a_tr for the strain form
                           * on the coarse grid): -1 (default) = the form of
                           * the levels above it (mid_form). */
    int nu_inc;           /* variable V-cycle (V_var, Sec. 5): level l runs
                           * nu1 + nu_inc (L - l) pre- and nu2 + nu_inc (L - l)
                           * post-smoothing steps, L the finest level;
                           * 0 (default) = the same count on every level. */
    int mid_form;         /* viscous form of the levels strictly between the
                           * finest and the coarsest inside V-cycles: -1
                           * (default) = the form of the call (Sec. 5 keeps
                           * the stencil form on the finer grids). */
    int merge_max_n;      /* kernel shapes (results are the same for every
                           * setting up to rounding order): levels with
                           * n <= merge_max_n cells per axis launch each
                           * colour phase of the smoother as one merged grid
                           * of bulk and special rows and the bulk rows of
                           * applies and residuals one vertex per thread;
                           * larger levels launch bulk and special rows
                           * separately, with the LDS-tiled right-hand-side
                           * passes and applies in 3D.  Default 64; 0
                           * selects the large-level kernels everywhere. */
    int spec_wide_min;    /* pressure special-row colour lists longer than
                           * this run in 256-thread workgroups, shorter ones
                           * in one-wave workgroups.  Default 65536. */
    int cycles;           /* V-cycles per preconditioner application inside
                           * iss_solve: z = the iterate after `cycles` steps
                           * of the stationary V-cycle iteration on K z = r
                           * from z = 0 (default 1). */
    double f16_rms;       /* ISS_FP32_FP16STORE: RMS the scaled input of
                           * the FP16 V-cycle is normalised to (default
                           * 2^-10: the cycle's corrections exceed its input
                           * by up to the inverse of the smallest eigenvalue,
                           * and FP16 ends at 65504). */
    int coarse_rhs_mod;   /* nonzero: when the coarsest level takes another
                           * form than the level above it, its right-hand
                           * side r_1 becomes r_1 + B^T M^-1 r_2, M the
                           * lumped (1/mu)-weighted pressure mass (Sec. 5,
                           * coarse grid solver; the paper's minus sign
                           * belongs to its opposite sign of B), folded
                           * into the coarse inverse at setup.  Default 0. */
    int bc;               /* boundary condition on the whole boundary of
                           * every level (eq. boundary): ISS_BC_NOSLIP
                           * (default) or ISS_BC_FREESLIP.  Free-slip fixes
                           * the normal velocity component on each face;
                           * the tangential components of boundary vertices
                           * are unknowns whose rows take the full element
                           * rows of the form (a_tr for ISS_INTERFACE, as
                           * Sec. 2.2 requires on Gamma_F).  Not with the
                           * learned band correction (iss_net_create). */
    int split_align;      /* kernel shape (results equal up to rounding
                           * order): the colour-split layout of the smoother
                           * stores each colour run of a row in q entries,
                           * q >= ceil((n+1)/(d+1)).  0 (default): q is
                           * rounded up to a multiple of 16 (FP64 runs on
                           * 128-byte lines) or else of 8 where that adds
                           * at most a quarter, otherwise unpadded; a value
                           * 1..64 rounds q up to a multiple of it on every
                           * level. */
    int coarse_solver;    /* ISS_COARSE_DIRECT (default): the bordered dense
                           * inverse of the coarsest level, factored on the
                           * host at first use.  ISS_COARSE_MINRES: the
                           * Krylov coarse solver of Sec. 5 -- MINRES on the
                           * coarsest level's system, block-diagonally
                           * preconditioned by minres_cg Jacobi-preconditioned
                           * CG steps on the velocity block and the lumped
                           * (1/mu-weighted) pressure mass, minres_iters
                           * steps from zero, with the constant pressure
                           * removed from its right-hand side and the
                           * weighted pressure mean from its result.  Sec. 5
                           * pairs it with the strain form on the coarse grid
                           * (coarse_form, coarse_rhs_mod): the CG needs a
                           * positive definite velocity block. */
    int minres_iters;     /* MINRES steps per coarse solve (default 30)     */
    int minres_cg;        /* CG steps per preconditioner application
                           * (default 5; 0: the Jacobi diagonal alone)      */
} iss_options;

typedef struct {
    int iterations;       /* V-cycles (= outer iterations) performed        */
    double relres;        /* final ||b - K x||_2 / ||b||_2 (FP64)           */
    double seconds;       /* wall time of the solve (host clock, synced)    */
    int history_len;      /* entries written to history                     */
    double* history;      /* optional host array (maxit+1) of relres, or 0  */
    int net_accepted;     /* band corrections kept by the safeguard          */
    int net_rejected;     /* band corrections dropped (plain V-cycle used)   */
} iss_solve_info;

/* Fill *opt with the defaults above.  Returns ISS_OK. */
int iss_default_options(iss_options* opt);

/* Create a problem: dim in {2, 3}; the unit cube (square) as macro^d
 * cubes x 6 Kuhn tetrahedra (squares x 2 triangles) refined `levels`
 * times (finest level: n = macro * 2^levels cells per axis), with
 * multigrid levels coarse_level..levels (coarse_level >= 1).  Viscosity
 * mu[phase] > 0 for phase 0..nphase-1 (nphase <= 254).  Setup (element
 * classification, interface lists, element tables, coarse factorisation)
 * runs on the host and device 0 of the current HIP device.
 * opt may be NULL for defaults.  *out receives the handle. */
int iss_problem_create(int dim, int macro, int levels, int coarse_level,
                       const iss_inclusion* inclusions, int ninclusions,
                       const double* mu, int nphase, const iss_options* opt,
                       iss_problem** out);
/* Same, with the viscosity given per fine element instead of by
 * inclusions (any geometry; Sec. 5 writes the system for a general
 * piecewise constant viscosity, the closing remark of Sec. 2.2 allows
 * interfaces that the mesh does not resolve).  elem_phase (host, read
 * during the call) holds one phase per element of the finest level,
 * phase < nphase: element (cell c, type t) at index c * T + t with
 * T = 6 (3D) or 2 (2D), cell c = ci + n (cj + n ck) for the cell with
 * lowest corner (ci, cj, ck), n = macro 2^levels; type t is the position
 * of the simplex's axis order in (x,y,z), (x,z,y), (y,x,z), (y,z,x),
 * (z,x,y), (z,y,x) (2D: (x,y), (y,x)), the order in which its edges from
 * the cell corner to the opposite corner step along the axes.  Coarse
 * levels need ISS_COARSE_MU_AVERAGE (ISS_E_INVAL otherwise). */
int iss_problem_create_elems(int dim, int macro, int levels, int coarse_level,
                             const uint8_t* elem_phase, const double* mu, int nphase,
                             const iss_options* opt, iss_problem** out);
void iss_problem_destroy(iss_problem* p);

/* Caller-owned workspace.  iss_workspace_bytes gives the bytes that every
 * call of p in precision prec needs for its work buffers: the V-cycle and
 * smoother vectors of every level in that precision, the FP64 FGMRES
 * arrays for the restart length of the options (2 restart + 3 vectors of
 * (dim+1) N doubles) and the two vectors of iss_asymptotic_rate, each
 * rounded up to 256 bytes.  Calls in several precisions need the sum over
 * those precisions.  iss_bind_workspace hands the library a device region
 * (256-byte aligned) to take these buffers from instead of hipMalloc; it
 * must come before the first call that needs a work buffer (ISS_E_INVAL
 * otherwise), stays owned by the caller, and must stay allocated until
 * iss_problem_destroy.  A call whose buffers no longer fit returns
 * ISS_E_NOWS.  Sizes follow the unknowns of the system of Sec. 5 on every
 * multigrid level. */
int iss_workspace_bytes(const iss_problem* p, int prec, size_t* bytes);
int iss_bind_workspace(iss_problem* p, void* dev_ptr, size_t bytes);

/* Number of lattice vertices N of `level` (a uniformly refined level of
 * the macro mesh, Sec. 2.2); a vector has (dim+1) N entries. */
int iss_num_vertices(const iss_problem* p, int level, int64_t* n);

/* Per-vertex class of `level` into host array cls (N bytes): bit 0 set for
 * interface vertices (incident element viscosities differ: the vertices
 * that keep the full a_tr rows in eq. equivalence-stencil, Sec. 2.2), bit 1
 * for boundary vertices.  Counts go to *ninterface / *nboundary if non-NULL. */
int iss_vertex_class(const iss_problem* p, int level, uint8_t* cls,
                     int64_t* ninterface, int64_t* nboundary);

/* Buoyancy load (the body force f of the Stokes problem of Sec. 1, eq. weaks
 * tested with the P1 basis): b = (0, .., 0, -rho sum_{T in buoyant phases}
 * |T|/(d+1), 0)
 * (body force (0,..,0,-rho) on elements of the listed phases) at `level`
 * into device FP64 vector b (overwritten).  With ISS_COARSE_MU_AVERAGE only
 * the finest level carries the problem's phases (ISS_E_INVAL otherwise). */
int iss_rhs_buoyancy(iss_problem* p, int level, const int* phases, int nbuoyant,
                     double rho, double* b, iss_stream_t stream);

/* Load of a body force given by its nodal values: b_k = M f_k for each
 * velocity component k, M the P1 mass matrix of `level` (the right-hand
 * side (f, v) of the weak form of Sec. 1 for the P1 interpolant of f),
 * fixed velocity entries and the pressure field zero.  f: device FP64,
 * d fields of N nodal values [f_1 | .. | f_d] (the caller evaluates f at
 * the vertices); b: device FP64 vector of (d+1) N entries, overwritten.
 * Sec. 4 forces the viscosity layers and columns with
 * f = (0, 0, -cos(2 pi x) cos(2 pi y) sin(pi z)). */
int iss_rhs_nodal_force(iss_problem* p, int level, const double* f, double* b,
                        iss_stream_t stream);

/* Stabilised P1-P0 discretisation on the finest level (Sec. 3): P1
 * velocity as above, one pressure per element, the interior-penalty
 * stabilisation of eq. stabc,
 *   c(p, q) = gamma sum_i 1/(2 mu_i) sum_{F interior to Omega_i}
 *             |T1||T2| / (|T1| + |T2|) [p]_F [q]_F,
 * (facets between elements of different viscosity and boundary facets are
 * not penalised) and b(v, q) = -(div v, q).  A P1-P0 vector holds the d
 * velocity fields of N entries followed by ne element pressures, element
 * e = c * T + t in the order of iss_problem_create_elems (c the cell, t the
 * type); fixed velocity entries as above.  iss_num_elements gives ne.
 * The calls need ne >= N (every 3D lattice; 2D lattices with n >= 3);
 * gamma > 0 (Sec. 4 takes gamma = 1).  Device FP64 vectors, caller-owned.
 *
 * iss_p1p0_apply: y = K x with K = [[A, B0^T], [B0, -C]], A the viscous
 * form `form` as in iss_apply (the discrete problem of Sec. 3 takes a_tr,
 * ISS_INTERFACE).
 * iss_p1p0_flux: the post-processed facet fluxes of Sec. 3, flux[e (d+1)
 * + a] = int_F u_h . n_T + gamma / (2 mu) |T||T'| / (|T| + |T'|)
 * (p_T - p_T') for the facet F of element T = e opposite its local vertex a
 * (local vertices in the order of the element's path through its cell,
 * the second term only on penalised facets); the fluxes of an element sum
 * to -(B0 u - C p)_T, zero for a solution of K x = (f, 0). */
int iss_num_elements(const iss_problem* p, int64_t* ne);
int iss_p1p0_apply(iss_problem* p, int form, double gamma, const double* x, double* y,
                   iss_stream_t stream);
int iss_p1p0_flux(iss_problem* p, double gamma, const double* x, double* flux, iss_stream_t stream);

/* y = K x (block ISS_FULL_STOKES) or y = (A x_u, 0) (ISS_VELOCITY_ONLY) at
 * `level` with the viscous form `form`: the saddle-point operator of the
 * system of Sec. 5 with A from eq. standard (strain), eq. newbil applied
 * as eq. equivalence-stencil (interface) or the gradient form of Sec. 1.
 * prec selects the element type of x and y (double, float, BF16 storage
 * with FP32 arithmetic); accumulation in the arithmetic type. */
int iss_apply(iss_problem* p, int form, int block, int level, int prec,
              const void* x, void* y, iss_stream_t stream);

/* r = b - K x at `level`, the residual of the system of Sec. 5 that the
 * multigrid cycle restricts and the solve monitors.  If norms is non-NULL
 * it receives d+2 FP64 numbers: the Euclidean norm of each field of r and
 * of all of r (the call then synchronises). */
int iss_residual(iss_problem* p, int form, int level, int prec, const void* x,
                 const void* b, void* r, double* norms, iss_stream_t stream);

/* nsteps Uzawa smoothing steps (eq. Uzawa_smooth) in place on x with
 * right-hand side b: symmetric multicolour Gauss-Seidel on the velocity
 * (colours (i+j+k) mod (d+1) forward with components 1..d, then the exact
 * reverse), then delta from one forward colour-ordered Gauss-Seidel sweep
 * on C started from 0 for B u - C p - g, and p += omega delta.  For the
 * gradient and interface forms, whose point-diagonal blocks are diagonal,
 * the first backward colour phase repeats an exact solve of the last
 * forward one and is skipped (a no-op in exact arithmetic). */
int iss_smooth(iss_problem* p, int form, int level, int prec, int nsteps,
               void* x, const void* b, iss_stream_t stream);

/* iss_smooth without any allocation, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  Arguments and results are those of
 * iss_smooth.  The colour-split copies of x and b and the smoother's work
 * fields, 3 (dim+1) Ns elements of the precision's size (Ns = the split
 * length of the level: (dim+1) ceil((n+1)/(dim+1)) (n+1)^(dim-1)), live in
 * one static device array of ISS_NOALLOC_SCRATCH_BYTES per GPU, held until
 * the process ends; a level that needs more returns ISS_E_INVAL (3D: up to
 * 65^3 in FP64, 2D: up to 513^2 in FP64).  The call makes no hipMalloc,
 * hipFree or other allocation; it must be made on the device current when
 * the problem was created (ISS_E_INVAL otherwise).  Every call on one GPU
 * uses that GPU's single array: calls that overlap on one GPU (several
 * streams, threads or problems) race and must be serialised by the caller.
 * The array keeps the last call's contents; the call clears what it needs
 * cleared itself. */
#define ISS_NOALLOC_SCRATCH_BYTES (32u << 20)
int iss_smooth_noalloc(iss_problem* p, int form, int level, int prec, int nsteps,
                       void* x, const void* b, iss_stream_t stream);

/* Same as iss_smooth, for measurement: HIP events recorded on `stream`
 * around every bulk velocity colour-phase launch and around every step.
 * ms[0] receives the average duration of one bulk velocity colour-phase
 * launch (interior isoviscous vertices of one colour class), ms[1] the
 * average duration of one whole step, in milliseconds.  Synchronises. */
int iss_smooth_timed(iss_problem* p, int form, int level, int prec, int nsteps,
                     void* x, const void* b, iss_stream_t stream, double* ms);

/* Grid transfers between `level` (fine) and level-1, the standard
 * transfers of the multigrid method of Sec. 5: restriction rc = P^T rf
 * (velocity zero on coarse boundary vertices) and xf += P ec, P = P1
 * interpolation between the nested lattices. */
int iss_restrict(iss_problem* p, int level, int prec, const void* rf, void* rc,
                 iss_stream_t stream);
int iss_prolong_add(iss_problem* p, int level, int prec, const void* ec, void* xf,
                    iss_stream_t stream);

/* Direct solve on the coarsest level (Sec. 5 allows a direct coarse
 * solver): x = K_c^+ b with sum_j w_j p_j = 0, w_j = int mu^{-1} lambda_j
 * (the space Q of Sec. 1).  FP64 always. */
int iss_coarse_solve(iss_problem* p, int form, const double* b, double* x,
                     iss_stream_t stream);

/* One V(nu1, nu2) cycle of the all-at-once Uzawa multigrid of Sec. 5
 * (smoother eq. Uzawa_smooth, standard transfers, direct coarsest solve)
 * on the finest level, in place on x.
 *
 * The part of the cycle below the finest level works only on the
 * library's own per-level buffers.  Its first run for a (coarse form,
 * precision) pair is eager; the second records it once as a HIP graph (on
 * an internal non-blocking stream) and every later cycle, here and inside
 * iss_solve, replays that graph on `stream`: the same kernels with the
 * same arguments, so the results are bitwise those of eager launches.
 * Setting ISS_VCYCLE_GRAPH=0 in the environment before iss_problem_create
 * keeps every launch eager; if recording fails the problem falls back to
 * eager launches by itself.  Cycles of one problem must not run
 * concurrently on several streams (they share the per-level buffers). */
int iss_vcycle(iss_problem* p, int form, int prec, void* x, const void* b,
               iss_stream_t stream);

/* Solve K x = b (the system of Sec. 5) on the finest level to
 * ||b - K x|| <= rtol ||b|| (the residual reduction of Sec. 5) from the
 * initial guess in x (FP64 vectors).  The outer iteration (options) is
 * Richardson with V-cycles (the stationary iteration of Sec. 5), or
 * right-preconditioned FGMRES (Saad 1993) with `cycles` stationary
 * V-cycles from zero as preconditioner.  prec = ISS_FP32 runs the V-cycle
 * (stencil applies, smoothers, transfers) in FP32 while the outer
 * residual, orthogonalisation, solution update and the coarsest solve
 * stay FP64; ISS_FP32_BF16STORE does the same with the V-cycle's vectors
 * stored in BF16, ISS_FP32_FP16STORE with them stored in FP16: FP16 has
 * five exponent bits, so that V-cycle runs on the symmetrically scaled
 * system (S K S) y = gamma S v, S = diag(sig_u on velocity, sig_p on
 * pressure) chosen at creation to make the isoviscous diagonal one for the
 * viscosity sqrt(mu_min mu_max), gamma making the RMS of gamma S v the
 * option f16_rms, and the preconditioned vector is S y / gamma.  info may
 * be NULL. */
int iss_solve(iss_problem* p, int form, int prec, double rtol, int maxit, double* x,
              const double* b, iss_solve_info* info, iss_stream_t stream);

/* Asymptotic convergence rate of the stationary V-cycle iteration, measured
 * as in Sec. 5 (the residual reduction per cycle of the homogeneous
 * problem after many cycles, the iterate rescaled every cycle).  x (FP64
 * device vector, velocity zero on the boundary) is the start and is
 * overwritten; each of the iters steps runs one FP64 V-cycle (options as
 * in iss_solve) on K x = 0 from x, removes the pressure mean (the
 * constant pressure spans the kernel of K and passes through the cycle
 * unchanged), and stores ||K x_new|| / ||K x|| in rates[step] (host array
 * of iters entries) before rescaling x to ||K x|| = 1.  The last entries
 * approach the asymptotic rate.  Synchronises every step. */
int iss_asymptotic_rate(iss_problem* p, int form, int iters, double* x, double* rates,
                        iss_stream_t stream);

/* y = a x + b y for FP64 device vectors of length n (the vector updates of
 * callers that drive the solver pieces themselves). */
int iss_axpby(double a, const double* x, double b, double* y, int64_t n, iss_stream_t stream);

/* Euclidean dot product of two FP64 device vectors of length n (the inner
 * products of the outer Krylov iteration). */
int iss_dot(iss_problem* p, const double* a, const double* b, int64_t n, double* out,
            iss_stream_t stream);

/* ---- learned interface-band correction (3D) --------------------------------
 * Not part of the paper: a small convolutional network that corrects the
 * V-cycle output on the band of vertices within Chebyshev distance 2 of an
 * interface vertex (finest level), where the plain smoother degrades.
 * Network: three 3x3x3 convolutions 8 -> 16 -> 16 -> 4 channels with ReLU,
 * no biases, zero padding off the band; BF16 operands with FP32
 * accumulation (MFMA).  Input channels per band vertex: r_1..r_3 / s_u,
 * r_p / s_p, log10(max incident viscosity) / 4, interface flag, 0, 0, where
 * s_u and s_p are the band RMS of the velocity and pressure residual.
 * Outputs are in Jacobi units: channel 0..2 times s_u / (6 mu h) and
 * channel 3 times s_p mu / (6 beta h^3), mu = largest incident viscosity,
 * form the correction; training targets are errors in the same units.
 * Parameters: FP32, flat [W1 | W2 | W3], W[c_out][c_in][tap], tap =
 * (dx+1) + 3 (dy+1) + 9 (dz+1); 12096 values. */
typedef struct iss_net iss_net;

/* Create the network state for the finest level of p (band, buffers).  The
 * network may outlive p: after iss_problem_destroy its input, forward,
 * target, backward and Adam calls still work, the calls that need the
 * problem (iss_net_correction, iss_problem_set_net) return ISS_E_INVAL. */
int iss_net_create(iss_problem* p, iss_net** out);
void iss_net_destroy(iss_net* net);
/* Band size M and parameter count. */
int iss_net_info(const iss_net* net, int64_t* band_size, int64_t* num_params);
/* Band vertex ids (ascending) into host array band (M entries). */
int iss_net_band(const iss_net* net, int32_t* band);
/* Load FP32 parameters from device memory (converted to BF16 fragments). */
int iss_net_set_weights(iss_net* net, const float* w, iss_stream_t stream);
/* Build the input from an FP64 residual r ((d+1) N, device); scales, if
 * non-NULL, receives (s_u, s_p) on the host (synchronises). */
int iss_net_features(iss_net* net, const double* r, double* scales, iss_stream_t stream);
/* Run the network on the current input; y (device, M x 4 FP32, band order)
 * receives the output if non-NULL. */
int iss_net_forward(iss_net* net, float* y, iss_stream_t stream);
/* Training targets from an error vector e ((d+1) N, FP64, device): t (M x 4
 * FP32) = e on the band in the output units above (current scales). */
int iss_net_targets(iss_net* net, const double* e, float* t, iss_stream_t stream);
/* Gradient with respect to the parameters (grad: device FP32, overwritten)
 * of the last forward pass.  With t non-NULL the loss is the mean squared
 * error against t (value to *loss on the host if non-NULL; synchronises);
 * with t NULL the output gradient set by iss_net_output_grad is used. */
int iss_net_backward(iss_net* net, const float* t, float* grad, double* loss, iss_stream_t stream);
/* The correction c ((d+1) N FP64, device, overwritten; zero off the band)
 * given by the last forward pass. */
int iss_net_correction(iss_net* net, double* c, iss_stream_t stream);
/* Set the output gradient dL/dy of the last forward pass from a gradient
 * with respect to the correction, dL/dc = factor * g (g: (d+1) N FP64,
 * device). */
int iss_net_output_grad(iss_net* net, const double* g, double factor, iss_stream_t stream);
/* One Adam step (beta 0.9 / 0.999, eps 1e-8, bias-corrected, step >= 1) on
 * n FP32 parameters w with moments m, v and gradient g (device). */
int iss_adam_step(int64_t n, float* w, float* m, float* v, const float* g, float lr, int step,
                  iss_stream_t stream);
/* Band rows of the network input set by iss_net_features (M x 8 BF16 bit
 * patterns, band order, device memory of the caller) out to dst, or back
 * in from src, so that training inputs can be stored compactly and
 * replayed without the residual they came from. */
int iss_net_save_input(iss_net* net, uint16_t* dst, iss_stream_t stream);
int iss_net_load_input(iss_net* net, const uint16_t* src, iss_stream_t stream);
/* Attach a network to iss_solve (NULL detaches).  With a network attached
 * the preconditioner is z = V(r) + c, c = the band correction computed from
 * r - K V(r), kept only if it lowers that residual's norm. */
int iss_problem_set_net(iss_problem* p, iss_net* net);

/* Kernel launches of the smoother and of the bulk apply/residual, counted
 * per kernel shape on the host at launch time (graph replays of the coarse
 * V-cycle are not counted).  Lets a caller confirm which kernel family
 * served a call. */
enum iss_launch_kind {
    ISS_L_VEL_RHS = 0,        /* g = f - B^T p, all interior rows          */
    ISS_L_GS_VEL_BULK,        /* velocity colour phase, bulk rows          */
    ISS_L_GS_VEL_SPECIAL,     /* velocity colour phase, special rows       */
    ISS_L_GS_VEL_MERGED,      /* velocity colour phase, bulk + special     */
    ISS_L_P_RHS_GROUPED,      /* s = B u - C p - g on large levels         */
    ISS_L_P_RHS_MERGED,       /* s pass merged with colour-0 special rows  */
    ISS_L_GS_P_BULK,          /* pressure colour phase, bulk rows          */
    ISS_L_GS_P_SPECIAL,       /* pressure special rows, one-wave groups    */
    ISS_L_GS_P_SPECIAL_WIDE,  /* pressure special rows, 256-thread groups  */
    ISS_L_GS_P_MERGED,        /* pressure colour phase, bulk + special     */
    ISS_L_APPLY_BULK,         /* apply / residual, bulk rows (small levels) */
    ISS_L_APPLY_TILED,        /* apply / residual, bulk rows, LDS z march   */
    ISS_L_KINDS
};
/* Copy the ISS_L_KINDS counters into counts (host, n >= ISS_L_KINDS
 * entries); reset != 0 then zeroes them. */
int iss_launch_counts(iss_problem* p, int64_t* counts, int n, int reset);

/* Message describing the last error on the calling thread. */
const char* iss_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* ISS_H */
