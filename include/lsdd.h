/*
 * lsdd.h — C-ABI of the MI355X LS-AMG-DD library (liblsdd.so).
 *
 * The library builds and applies the least-squares AMG-DD multilevel
 * preconditioner for an SPD matrix given in Gram form A = G^T G, where G stacks
 * element-local Gram factors of a conforming finite-element assembly
 * (Krzysik, Southworth, Wimmer: Sec. 2 for the method, Prop. "elementwise Gram
 * formulation" of Sec. 5.1 for A = sum_T R_T^T A_T R_T = G^T G, Sec. 5.2 for the
 * eigendecomposition factor G_T = Lambda_+^{1/2} Q_+^T), and solves A x = b with
 * preconditioned CG whose preconditioner is one symmetric V-cycle.
 *
 * Conventions for every entry point:
 *  - Every function returns an lsdd_status; no C++ exception crosses the ABI.
 *    On failure lsdd_last_error() returns a thread-local message.
 *  - Integer index arrays are 0-based.  Dense element blocks are row-major
 *    (they are symmetric, so the order only matters for the asymmetry check).
 *  - Buffers flagged "device" are HIP device pointers on the current device;
 *    buffers flagged "host" are ordinary host memory.
 *  - All device work is enqueued on the caller's hip stream (`hip_stream`,
 *    a hipStream_t cast to void*; NULL = the null stream).  A function returns
 *    after the work it must report on (status, iteration counts) is complete.
 *  - Input arrays are caller-owned and are copied during setup; the hierarchy
 *    owns all of its device memory until lsdd_destroy().
 *  - Index validation happens on the host before any kernel launch.
 *  - A hierarchy is not thread-safe; use one handle per host thread.
 */
#ifndef LSDD_H
#define LSDD_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    LSDD_OK = 0,
    LSDD_E_INVAL = 1,        /* bad argument, index out of range, asymmetric block, NaN/Inf   */
    LSDD_E_NOT_SPSD = 2,     /* an element block has lambda_min < -spsd_tol * lambda_max     */
    LSDD_E_NOMEM = 3,        /* device or host allocation failed                              */
    LSDD_E_HIP = 4,          /* a HIP runtime call failed                                     */
    LSDD_E_NOCONV = 5,       /* PCG reached max_iter; x holds the last iterate                */
    LSDD_E_BREAKDOWN = 6,    /* PCG breakdown (p^T A p <= 0 or a non-finite scalar)            */
    LSDD_E_UNSUPPORTED = 7,  /* a size or option this build does not handle                   */
    LSDD_E_NUMERIC = 8       /* a local factorisation failed (a local matrix is not SPD)      */
} lsdd_status;

typedef struct lsdd_hierarchy lsdd_hierarchy;   /* opaque, library-owned */

/* Setup and solve parameters.  Paper defaults (Sec. 6): two passes of standard
 * aggregation, tau_cut = tau_const * max_j mult(j) (eq. tau-cut), at most three
 * levels, stop below 10 DOFs or above 25 % density; the build adds the outer
 * PCG tolerance and the precision of the cycle. */
typedef struct {
    int32_t max_levels;         /* level cap (>= 1); default 3                                */
    int32_t agg_passes;         /* standard-aggregation passes on level 0; default 2          */
    int32_t agg_passes_coarse;  /* passes on coarser levels; default 1                        */
    int32_t modes_fixed;        /* > 0: keep this many smallest mu per aggregate; 0: tau_cut   */
    int32_t min_coarse;         /* a level with fewer DOFs is the coarsest; default 10         */
    int32_t max_iter;           /* PCG iteration cap; default 1000                             */
    int32_t precision;          /* cycle precision at setup (FP64 PCG outside in all cases):
                                   0 = FP64 cycle; 1 = FP32 cycle (FP32 copies of the operator,
                                   subdomain inverses and transfers are kept); 2 = as 1, plus
                                   FP32 copies of the subdomain factors X = L^{-1} for the mixed
                                   cycle (see lsdd_set_cycle_precision)                      */
    int32_t blocked_eig_min;    /* local spectral problems with |omega| >= this use the blocked
                                   multi-workgroup tridiagonal reduction; 0 = library default
                                   (192), < 0 = never; values below 66 act as 66            */
    int32_t closure;            /* overlaps: 0 = G-row closure (Def. "G-row closure", default);
                                   1 = algebraic A-closure (Def. "algebraic A-closure"), the
                                   comparison of Sec. 5.3: Omega_i = omega_i plus the DOFs p
                                   with an entry |A(p,q)| > closure_tol sqrt(A(p,p) A(q,q)),
                                   q in omega_i; the local matrix is the G-row closure's
                                   A~_Omega cut down to those DOFs                          */
    int32_t smoother;           /* block Schwarz smoother M^{-1} of the cycle (Sec. 2; the
                                   post-smoother is M^{-T}): 0 = multiplicative Schwarz on the
                                   overlaps, colour-major forward, reverse after the coarse
                                   correction (default, Sec. 6); 1 = restricted additive
                                   Schwarz (local solves on the overlaps, corrections kept on
                                   the aggregates; M^{-T} restricts the residual instead);
                                   2 = block Jacobi on the aggregates (A_ww^{-1})            */
    int32_t elem_factor;        /* element Gram factor (Sec. 5.2): 0 = Lambda_+^{1/2} Q_+^T from
                                   the eigendecomposition (default); 1 = pivoted Cholesky
                                   (largest remaining diagonal pivot, stop at rank_rtol or
                                   n_T eps times max diag; a remainder above that bound ->
                                   LSDD_E_NOT_SPSD).  Under full-support rows the hierarchy
                                   does not depend on the choice (Galerkin products up to
                                   rounding)                                                */
    int32_t galerkin_precision; /* Galerkin products G_T P_T and A_g = Y^T Y of levels >= 1
                                   (Sec. 2, Galerkin Gram recursion): 0 = FP64 matrix cores
                                   (default); 1 = FP32 matrix cores, operands rounded to FP32,
                                   FP32 accumulation (the coarse operators then carry FP32
                                   rounding; local spectral problems, coarsest factorisation
                                   and PCG stay FP64)                                        */
    double tau_const;           /* tau_cut = tau_const * max mult; default 0.75               */
    double max_density;         /* nnz(A_l)/n_l^2 above this -> coarsest; default 0.25         */
    double rtol;                /* PCG stop: ||r||_2 <= rtol ||b||_2; default 1e-8              */
    double cluster_tol;         /* complete an eigenvalue cluster cut at its edge; 1e-9        */
    double band_tol;            /* mu within band_tol above 1/tau_cut is retained; 1e-9        */
    double rank_rtol;           /* element rank tolerance / lambda_max; 0 = n_T * eps          */
    double spsd_tol;            /* lambda_min < -spsd_tol lambda_max -> LSDD_E_NOT_SPSD; 1e-12 */
    double closure_tol;         /* relative size below which an entry of A counts as zero for
                                   the A-closure; default 1e-12                               */
} lsdd_params;

/* Per-solve report (one per right-hand side). */
typedef struct {
    int32_t iters;              /* PCG iterations = applications of A                         */
    int32_t converged;          /* 1 if ||r|| <= rtol ||b||                                    */
    double rel_res;             /* final ||r||_2 / ||b||_2 (recurrence residual)               */
    double setup_s;             /* wall time of the setup that built the hierarchy             */
    double solve_s;             /* wall time of this solve                                     */
} lsdd_info;

/* Fill *p with the defaults listed above. */
void lsdd_params_default(lsdd_params* p);

/* Build a hierarchy from element blocks and their DOF cover (Def. "DOF cover",
 * Prop. "elementwise Gram formulation").
 *   n            number of global DOFs (1 <= n < 2^31)
 *   n_elem       number of elements (>= 1)
 *   elem_ptr     host, int64[n_elem+1]: element e owns elem_dofs[elem_ptr[e] .. elem_ptr[e+1])
 *   elem_dofs    host, int32[elem_ptr[n_elem]]: global DOFs, distinct within an element;
 *                every DOF must belong to at least one element; 1 <= n_T <= 128
 *   elem_blocks  host or device (mem_is_device), float64, the n_T x n_T blocks
 *                concatenated, row-major; each must be symmetric and SPSD
 *   node_of_dof  host, int32[n] or NULL: supernode of each DOF (all components of a
 *                vertex, the DOFs of one edge, ...); supernodes are the vertices of
 *                the aggregation graph.  NULL = every DOF is its own supernode
 *   agg_of_dof   host, int32[n] or NULL: caller-given level-0 aggregates (values
 *                0..n_agg-1, each used); NULL = standard aggregation
 *   params       NULL = defaults
 * Returns LSDD_E_NOT_SPSD (message names the element) for an indefinite block,
 * LSDD_E_INVAL for bad indices or an asymmetric block. */
lsdd_status lsdd_setup_elements(int64_t n, int64_t n_elem, const int64_t* elem_ptr,
                                const int32_t* elem_dofs, const double* elem_blocks,
                                const int32_t* node_of_dof, const int32_t* agg_of_dof,
                                int mem_is_device, const lsdd_params* params, void* hip_stream,
                                lsdd_hierarchy** out);

/* Build ONE hierarchy for a batch of independent problems: the method applied
 * to their block-diagonal union (Sec. 2: aggregates, overlaps, colours and coarse
 * spaces of different instances never meet, so the union's hierarchy restricted
 * to an instance is that instance's own hierarchy).  Every setup and cycle kernel
 * then runs over all instances at once; lsdd_solve runs one CG recurrence per
 * (instance, right-hand side) pair.
 *   n_inst       number of instances (>= 1)
 *   inst_n       host, int64[n_inst]: DOFs of instance i (>= 1)
 *   inst_n_elem  host, int64[n_inst]: elements of instance i (>= 1); the element
 *                arrays list the elements of instance 0 first, then instance 1, ...
 *   elem_ptr     host, int64[sum inst_n_elem + 1], elem_ptr[0] = 0
 *   elem_dofs    host, int32: instance-local DOF indices (0 .. inst_n[i]-1)
 *   elem_blocks  host or device (mem_is_device), float64 blocks as in lsdd_setup_elements
 *   node_of_dof  host, int32[sum inst_n] or NULL: instance-local supernode ids, instances
 *                concatenated (each instance uses 0..count-1)
 *   agg_of_dof   host, int32[sum inst_n] or NULL: instance-local level-0 aggregates, concatenated
 * DOF j of instance i is DOF inst_off[i] + j of the union (inst_off = prefix sums of
 * inst_n), which is also the layout of b and x in lsdd_solve; lsdd_segments returns
 * inst_off.  Per instance: tau_cut uses the instance's own largest multiplicity and the
 * stopping tests (max_levels, min_coarse, max_density) are applied to the instance's
 * own level, so every instance gets the hierarchy it would get alone; an instance whose
 * hierarchy ends on level l is solved there with the dense inverse of its block of A_l
 * while the others continue (lsdd_level_segments).  An instance that retains no mode
 * on a level while others do -> LSDD_E_UNSUPPORTED. */
lsdd_status lsdd_setup_batched(int32_t n_inst, const int64_t* inst_n, const int64_t* inst_n_elem,
                               const int64_t* elem_ptr, const int32_t* elem_dofs, const double* elem_blocks,
                               const int32_t* node_of_dof, const int32_t* agg_of_dof, int mem_is_device,
                               const lsdd_params* params, void* hip_stream, lsdd_hierarchy** out);

/* As lsdd_setup_elements with element coefficients: the blocks passed are the
 * unit blocks A_e^(1) and the hierarchy is built for A_e = theta_e A_e^(1)
 * (elem_scale = theta, float64[n_elem], host or device like the blocks; NULL =
 * all ones).  theta is kept for lsdd_update_theta. */
lsdd_status lsdd_setup_elements_scaled(int64_t n, int64_t n_elem, const int64_t* elem_ptr,
                                       const int32_t* elem_dofs, const double* elem_blocks,
                                       const double* elem_scale, const int32_t* node_of_dof,
                                       const int32_t* agg_of_dof, int mem_is_device,
                                       const lsdd_params* params, void* hip_stream, lsdd_hierarchy** out);

/* Replace the level-0 operator by A(theta') = sum_e theta'_e A_e^(1) (theta' device
 * float64[n_elem]) while keeping the rest of the hierarchy: later solves run PCG on
 * A(theta') preconditioned by the cycle built for the setup's theta (its level-0
 * residuals use A(theta')).  Meant for nearby theta' (finite differences); passing
 * the setup's theta restores the original operator bit for bit.
 * LSDD_E_UNSUPPORTED for a hierarchy built from a CSR Gram factor. */
lsdd_status lsdd_update_theta(lsdd_hierarchy* h, const double* theta, void* hip_stream);

/* Element bilinear forms out[e] = scale * sum_k u_{k,S_e}^T B_e v_{k,S_e} over nrhs
 * pairs of vectors (all device pointers but elem_ptr): with scale = -1, u_k the
 * adjoint solutions lambda_k and v_k the solutions u_k, this is the gradient
 * dL/dtheta_e = -sum_k lambda_{k,e}^T A_e^(1) u_{k,e} of u = A(theta)^{-1} b for
 * element blocks linear in their coefficient (Sec. 5.1, elementwise assembly).
 *   elem_ptr   host int64[n_elem + 1] (elem_ptr[0] = 0, element sizes 1 .. 4096);
 *              elem_dofs device int32 (indices < ld, not checked); blocks device
 *              float64, the n_e x n_e blocks row-major, concatenated
 *   u, v       device float64[nrhs * ld]: vector k at offset k * ld
 *   nrhs >= 1, ld >= 1; out device float64[n_elem] (overwritten)
 * Allocates two small device arrays per call (elem_ptr and the block offsets);
 * blocks until the result is written. */
lsdd_status lsdd_elem_bilinear(int64_t n_elem, const int64_t* elem_ptr, const int32_t* elem_dofs,
                               const double* blocks, const double* u, const double* v, int32_t nrhs,
                               int64_t ld, double scale, double* out, void* hip_stream);

/* For callers that cannot allocate device memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc): the same contraction as
 * lsdd_elem_bilinear, same arguments and result (identical kernels), with its
 * staging (elem_ptr and the block offsets) in a static device array of the library
 * instead of per-call allocations.  That array holds 2 (n_elem + 1) int64 entries
 * for at most 1,048,576 elements (16 MiB per GPU, held until the process ends);
 * n_elem above that -> LSDD_E_UNSUPPORTED before any device work.  Every call on
 * one GPU uses that GPU's copy of the array: calls that overlap on one GPU (other
 * threads, other streams) race.  Calls no hipMalloc/hipFree; blocks until the
 * result is written. */
lsdd_status lsdd_elem_bilinear_noalloc(int64_t n_elem, const int64_t* elem_ptr, const int32_t* elem_dofs,
                                       const double* blocks, const double* u, const double* v, int32_t nrhs,
                                       int64_t ld, double scale, double* out, void* hip_stream);

/* Build a hierarchy from a black-box sparse Gram factor G (m x n, CSR), the input
 * of Sec. 2 (A = G^T G, m >= n, full column rank).  Each row of G is its own cover
 * member: row j contributes g_j g_j^T with support = its stored pattern (all
 * stored entries count as support, zero values included).  Rows with no stored
 * entries are dropped (Sec. 2, after eq. row_multiplicity).
 *   rowptr  int64[m + 1], rowptr[0] = 0, non-decreasing; col int32[rowptr[m]] in
 *           [0, n); val float64[rowptr[m]]; a row holds at most 128 entries
 *   mem_is_device  0: rowptr, col, val are host arrays; 1: device arrays (the
 *           pattern is copied to the host once to build the cover; the values
 *           stay on the device, where the element factors and blocks are formed)
 *   node_of_dof, agg_of_dof  host, as in lsdd_setup_elements
 * The caller keeps ownership of every array.  A column with no entry (A
 * singular), a bad index or a non-finite value -> LSDD_E_INVAL; a row above 128
 * entries -> LSDD_E_UNSUPPORTED. */
lsdd_status lsdd_setup_gram_csr(int64_t m, int64_t n, const int64_t* rowptr, const int32_t* col,
                                const double* val, const int32_t* node_of_dof,
                                const int32_t* agg_of_dof, int mem_is_device, const lsdd_params* params,
                                void* hip_stream, lsdd_hierarchy** out);

/* Solve A x = b for nrhs right-hand sides with PCG (x0 = 0) preconditioned by
 * one V-cycle per iteration.  Every (segment, right-hand side) pair runs its own
 * CG recurrence (its own step lengths and stopping test, Hestenes-Stiefel beta;
 * with the FP32 cycle the flexible beta (r_new - r_old)^T z_new / r_old^T z_old);
 * a hierarchy built by lsdd_setup_elements has one segment, a batched one has one
 * per instance (lsdd_segments).  Right-hand sides are processed in blocks of 8
 * whose vectors are interleaved per DOF, so every operator byte of a cycle serves
 * all right-hand sides of the block.
 *   b, x   device, float64[nrhs * n] (right-hand side r at offset r*n); x is overwritten
 *   info   host, lsdd_info[nrhs * n_seg] or NULL; entry r * n_seg + s is pair (s, r)
 * NaN/Inf in b -> LSDD_E_INVAL.  LSDD_E_NOCONV leaves the last iterates in x. */
lsdd_status lsdd_solve(lsdd_hierarchy* h, const double* b, double* x, int32_t nrhs,
                       void* hip_stream, lsdd_info* info);

/* Solve with several separately built hierarchies: hs[i] x_i = b_i for i < n_inst,
 * each exactly as lsdd_solve with nrhs right-hand sides, run one after the other on
 * the stream.  (Uneven instances in single launches are the union hierarchy of
 * lsdd_setup_batched solved by one lsdd_solve.)
 *   hs     host array of n_inst hierarchy handles
 *   b, x   host arrays of n_inst device pointers, b[i], x[i] float64[nrhs * n_i]
 *   info   host, lsdd_info[n_inst * nrhs * n_seg_i] concatenated in instance order, or NULL
 * Stops at the first instance whose solve fails and returns its status. */
lsdd_status lsdd_solve_batched(int32_t n_inst, lsdd_hierarchy* const* hs, const double* const* b,
                               double* const* x, int32_t nrhs, void* hip_stream, lsdd_info* info);

/* Standalone V-cycle iteration, the solver mode of the paper's experiments (Sec. 6):
 * x_{k+1} = x_k + V(b - A x_k), where V is one symmetric V-cycle (forward
 * multiplicative Schwarz pre-smoothing, coarse correction, reverse-order
 * post-smoothing), until ||b - A x_k||_2 <= rtol ||b - A x_0||_2 (rtol and the
 * iteration cap max_iter from the parameters or lsdd_set_solve_params; the
 * paper uses rtol = 1e-10).  Runs in the hierarchy's cycle precision.
 *   b      device, float64[nrhs * n] (b = 0 is allowed: the iteration then
 *          drives x_0 to zero, as in the closure comparison of Sec. 5.3)
 *   x      device, float64[nrhs * n]: the initial iterates x_0 on entry (NOT
 *          zeroed), the last iterates on return
 *   info   host, lsdd_info[nrhs] or NULL: iters = cycles applied, rel_res =
 *          ||b - A x||_2 / ||b - A x_0||_2 (0 and converged when r_0 = 0)
 * Only hierarchies with one segment (not lsdd_setup_batched) -> else
 * LSDD_E_UNSUPPORTED; NaN/Inf in b or x_0 -> LSDD_E_INVAL; the cap reached ->
 * LSDD_E_NOCONV with the last iterates in x; a non-finite residual ->
 * LSDD_E_BREAKDOWN. */
lsdd_status lsdd_solve_stationary(lsdd_hierarchy* h, const double* b, double* x, int32_t nrhs,
                                  void* hip_stream, lsdd_info* info);

/* Switch the cycle precision of an existing hierarchy:
 *   0 = FP64 cycle;
 *   1 = FP32 cycle: FP32 vectors, operator entries, explicit subdomain inverses and
 *       transfers (needs a hierarchy set up with precision >= 1);
 *   2 = mixed cycle: FP32 vectors and transfers, subdomain solves as X^T (X r) with
 *       FP32 factors X = L^{-1} of A_Omega (symmetric positive semidefinite under
 *       rounding), residuals from the FP64 operator entries with FP64 sums (needs
 *       precision = 2; multiplicative Schwarz smoother and single right-hand sides
 *       only, else LSDD_E_UNSUPPORTED).  This is the variant for operators whose
 *       spectrum FP32 cannot resolve, e.g. a mass term 1e-8 below the div term.
 * The coarsest (terminal) solve and PCG stay FP64 in every mode; modes 1 and 2 use
 * flexible PCG.  LSDD_E_INVAL if the setup precision does not allow the mode. */
lsdd_status lsdd_set_cycle_precision(lsdd_hierarchy* h, int32_t precision);

/* Change the PCG stopping tolerance and iteration cap of an existing hierarchy. */
lsdd_status lsdd_set_solve_params(lsdd_hierarchy* h, double rtol, int32_t max_iter);

/* on != 0: run each PCG iteration as two replays of HIP graphs captured on the
 * first solve (operator apply, step and residual update, stopping test; then the
 * V-cycle, the new search direction); on = 0: launch every kernel directly.  The
 * results are bitwise the same either way.  Graphs need a non-NULL stream and are
 * not used while lsdd_trace is on; they are re-captured after parameter changes. */
lsdd_status lsdd_set_graph(lsdd_hierarchy* h, int32_t on);

/* Segments of the level-0 vector (host outputs, either may be NULL):
 *   n_seg     number of segments (1, or the instance count of a batched hierarchy)
 *   seg_off   int64[n_seg + 1]: segment s is DOFs [seg_off[s], seg_off[s+1]) */
lsdd_status lsdd_segments(const lsdd_hierarchy* h, int32_t* n_seg, int64_t* seg_off);

/* Instances on level l of a batched hierarchy (host outputs, either may be NULL):
 *   inst_off  int64[n_seg + 1]: instance i owns DOFs [inst_off[i], inst_off[i+1]) of
 *             level l (empty once its hierarchy has ended on a finer level)
 *   terminal  int32[n_seg]: 1 if instance i's hierarchy ends on level l (its block of
 *             A_l is solved directly there; it owns no aggregate on level l) */
lsdd_status lsdd_level_segments(const lsdd_hierarchy* h, int32_t level, int64_t* inst_off, int32_t* terminal);

/* Autotuner: on this hierarchy, time every candidate of the per-level launch
 * shapes with HIP events (the fastest of five runs after a warm-up, on the level's own
 * operators) and keep the fastest: CSR lanes per row of the residual kernel (8, 16,
 * 32 or 64 for single vectors; for blocks 4, 8 or 16 lanes that each hold all 8
 * right-hand sides of one nonzero slot, or 32 or 64 lanes split over (slot,
 * right-hand side)), tiles per work item of the
 * tiled subdomain product of the large overlaps (2, 4 or 8) and threads per DOF of
 * its finalize (8 or 32).  For single vectors on level 0 of a hierarchy built from
 * element blocks (at most 128 DOFs each) it also times the full products A x (the
 * residual before restriction and the PCG product) from the CSR against the
 * element-batch form A x = sum_e R_e^T (A_e x_e) (Sec. 2) with the packed lower
 * triangles of the A_e, built on the first call (one FP64 triangle per element, plus
 * an FP32 copy when the hierarchy has an FP32 cycle), and keeps the faster; on levels
 * whose rows share per-supernode column lists it times the CSR kernels with and
 * without them, and the sweep residuals by supernode row blocks
 * (1, 2 or 4 waves per run of up to 8 sweep rows of one supernode, x gathered once
 * per run and wave; another order of the cross-lane sums); in the mixed cycle it times the factor product with and without its
 * tile rows kept in LDS.  block
 * != 0 tunes the shapes of the 8-right-hand-side blocks, 0 those of single vectors,
 * for the current cycle precision.  The choice changes only the summation order of
 * the sums involved. */
lsdd_status lsdd_autotune(lsdd_hierarchy* h, int32_t block, void* hip_stream);

/* Launch shapes of level l (host int32[7]): CSR lanes per row for single vectors,
 * for blocks, tiles per work item, finalize threads per DOF, full products of single
 * vectors from the element triangles (1) or the CSR (0), whether the CSR kernels
 * read one shared column list per supernode (1) instead of a column index per entry
 * (0; available where the level's pattern is built on supernodes, i.e. every row of
 * a supernode has the same columns; same results) -- 2, 3, 4: the lists as with 1,
 * and the single-vector sweep residuals by supernode row blocks of 1, 2 or 4 waves
 * (where the level has sweeps); with 4, 8 or 16 lanes for blocks, the block sweep
 * residuals by row blocks too, with the same results as per row --, and whether the mixed cycle's
 * factor product keeps each tile row in LDS between its two passes (1) or reads it
 * again through the caches (0; same results). */
lsdd_status lsdd_level_tuning(const lsdd_hierarchy* h, int32_t level, int32_t* out);

/* Set the launch shapes of level l (host int32[7], the layout of lsdd_level_tuning),
 * e.g. to restore what lsdd_autotune chose for another cycle precision.  Every value
 * must be one of the autotuner's candidates (else LSDD_E_INVAL, nothing changed);
 * tiles per work item is ignored on the coarsest level; element products on a level
 * other than 0, on a hierarchy without element blocks or with an element above 128
 * DOFs, or shared column lists (row blocks) on a level without them ->
 * LSDD_E_UNSUPPORTED (the
 * triangles are built on first use).  Captured PCG graphs are
 * dropped and recaptured on the next solve.  Like lsdd_autotune, it changes only the
 * summation order of the sums involved. */
lsdd_status lsdd_set_level_tuning(lsdd_hierarchy* h, int32_t level, const int32_t* in);

/* Per-kernel timing: on != 0 clears the counters and records a pair of HIP
 * events on the solve stream around every launch of the traced kernel classes
 * (csr_resid_rows, sub_symv, sub_finalize, small_sub, csr_spmv, restrict,
 * prolong, coarse_symv, pcg_spmv); on = 0 stops recording.  lsdd_trace_get reads class idx
 * (0-based; LSDD_E_INVAL past the end): name (host char[name_len]), launches,
 * summed event time in ms and summed algorithmic bytes of those launches (the
 * bytes each launch must move at minimum: matrix entries, indices and vector
 * entries read or written once). */
lsdd_status lsdd_trace(lsdd_hierarchy* h, int32_t on);
lsdd_status lsdd_trace_get(lsdd_hierarchy* h, int32_t idx, char* name, int32_t name_len, int64_t* launches,
                           double* ms, double* bytes);

/* Apply the preconditioner once: z = V(r) (the symmetric V-cycle of Sec. 2 with
 * forward multiplicative Schwarz pre-smoothing and reverse-order post-smoothing).
 *   r, z   device, float64[n] */
lsdd_status lsdd_vcycle(lsdd_hierarchy* h, const double* r, double* z, void* hip_stream);

/* y = A_l x on level l (A_0 = A, A_{l+1} = P_l^T A_l P_l), from the CSR or, where the
 * level's tuning selects them, the element triangles.  x, y device float64[n_l]. */
lsdd_status lsdd_apply(lsdd_hierarchy* h, int32_t level, const double* x, double* y,
                       void* hip_stream);

/* Level summary (host outputs, any may be NULL):
 *   levels            number of levels L
 *   n_l, nnz_l        int64[L] each (structural nonzeros of A_l)
 *   oc, gc            operator complexity sum nnz_l / nnz_0, grid complexity sum n_l / n_0
 *                     (the complexity measures of Sec. 6) */
lsdd_status lsdd_hierarchy_info(const lsdd_hierarchy* h, int32_t* levels, int64_t* n_l,
                                int64_t* nnz_l, double* oc, double* gc);

/* Sizes of the arrays lsdd_export_level fills for level l (host int64[8]):
 *   [0] n_l  [1] nnz(A_l)  [2] n_agg (0 on the coarsest level)  [3] sum |omega_i| * k_i
 *   [4] sum |Omega_i|  [5] number of colours  [6] n_{l+1}  [7] number of elements on level l */
lsdd_status lsdd_level_sizes(const lsdd_hierarchy* h, int32_t level, int64_t* sizes);

/* Copy level-l data to host buffers (any may be NULL; sizes from lsdd_level_sizes):
 *   agg_of_dof int32[n_l] (-1 on the DOFs of instances whose hierarchy ends on level l); k int32[n_agg] (retained modes); Z float64[sum |w_i| k_i]
 *   (aggregate-major, each Z_i row-major |omega_i| x k_i, rows in ascending DOF order,
 *   columns in ascending mu); mu float64[sum |omega_i|] (sorted local spectra);
 *   colors int32[n_agg]; rowptr int64[n_l+1], col int32[nnz], val float64[nnz] (A_l, CSR,
 *   sorted columns); omega_sizes int32[n_agg] (|Omega_i|). */
lsdd_status lsdd_export_level(const lsdd_hierarchy* h, int32_t level, int32_t* agg_of_dof,
                              int32_t* k, double* Z, double* mu, int32_t* colors,
                              int64_t* rowptr, int32_t* col, double* val, int32_t* omega_sizes);

/* Level-0 element Gram factors (Sec. 5.2): ranks int32[n_elem] and, if G is not
 * NULL, float64[sum n_T^2] with G_T stored row-major as an n_T x n_T array whose
 * first r_T rows hold Lambda_+^{1/2} Q_+^T (remaining rows zero). */
lsdd_status lsdd_export_gram(const lsdd_hierarchy* h, int32_t* ranks, double* G);

/* Element Gram factors of level l (host outputs, any may be NULL).  Level 0: the
 * factors lsdd_export_gram returns.  Level l >= 1: the elements are the coarse
 * element groups (finer-level elements summed over the set of aggregates they
 * touch), and the factors are Gram rows of their summed blocks A_g (Sec. 5.1,
 * the remark that sums of element Grams are Grams of the coarser scale), from a
 * diagonally pivoted Cholesky factorization of each block (Sec. 5.2; pivot = the
 * largest remaining diagonal entry, lowest index among equal ones), truncated
 * when that entry is at most n_g eps max diag(A_g).  They replace the rows G P
 * (one per level-0 row) by rank(A_g) rows per group, and A_l = sum_g R_g^T
 * G_g^T G_g R_g up to the truncation.  The first call on a coarse level factors
 * its blocks on the device and keeps the result in the hierarchy.
 *   elem_ptr int64[n_e + 1], elem_dofs int32[elem_ptr[n_e]] (level-l DOFs of every
 *   element; n_e from lsdd_level_sizes); ranks int32[n_e]; G float64[sum n_g^2]
 *   with G_g stored row-major as an n_g x n_g array whose first r_g rows hold the
 *   factor rows (remaining rows zero).
 * Errors: LSDD_E_INVAL for a NULL hierarchy or a level out of range; device errors. */
lsdd_status lsdd_export_gram_level(lsdd_hierarchy* h, int32_t level, int64_t* elem_ptr, int32_t* elem_dofs,
                                   int32_t* ranks, double* G);

/* Library allocator hook (e.g. a framework's caching allocator).  alloc returns a
 * device pointer of at least `bytes` bytes on the current device or NULL; free
 * releases it.  NULL functions restore hipMalloc/hipFree.  Call before setup. */
typedef void* (*lsdd_alloc_fn)(uint64_t bytes, void* ctx);
typedef void (*lsdd_free_fn)(void* ptr, void* ctx);
void lsdd_set_allocator(lsdd_alloc_fn alloc, lsdd_free_fn free_fn, void* ctx);

/* Thread-local text of the last error ("" if none). */
const char* lsdd_last_error(void);

/* Release the hierarchy and all of its device memory.  NULL is accepted. */
lsdd_status lsdd_destroy(lsdd_hierarchy* h);

#ifdef __cplusplus
}
#endif

#endif /* LSDD_H */
