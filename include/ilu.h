/*
 * ilu.h -- C-ABI of libilu: matrix-free ILU(0) smoothing on uniformly refined
 * macro-tetrahedra (Drzisga, Wagner, Wohlmuth, "A matrix-free ILU realization
 * based on surrogates", arXiv:2210.15280), for AMD Instinct MI355X (gfx950).
 *
 * Problem (Sec. 2.1 and Sec. 3): for each macro-tetrahedron t with vertices
 * v1..v4 (their order fixes the DOF ordering), refinement level L >= 2
 * (n = 2^L intervals per edge) and a scalar coefficient kappa, let A be the
 * P1 stiffness matrix of a(u,v) = int grad(u) . kappa grad(v) restricted to
 * the N = C(n-1,3) interior lattice points (homogeneous Dirichlet values on
 * the macro boundary), and L D L^T its ILU(0) in lexicographic order.  A
 * smoothing step is the Richardson step
 *     x <- x + C^{-1} (b - A x),   C = L D L^T,
 * where C is either the exact ILU(0) (stored factors) or its surrogate: one
 * polynomial per lower stencil direction for L and one for 1/D, fitted by
 * least squares on the sample sets S_d (Sec. 4.1), evaluated on the fly
 * (Alg. 2), with the boundary variant V2 or V1 (ilu_opts.boundary).
 *
 * Vectors at this interface: FP64 device arrays, interior points of each
 * tetrahedron in lexicographic order (z slowest, then y, then x; x,y,z >= 1,
 * x+y+z <= n-1), tetrahedra concatenated in the order given to
 * ilu_setup_surrogate; ilu_layout reports each tetrahedron's offset.
 *
 * Conventions: every call returns ILU_OK (0) or a negative error code; no
 * exception crosses the interface and nothing is printed.  Device pointers
 * are caller-owned; the handle owns every buffer it allocates.  `hip_stream`
 * is a hipStream_t (NULL = default stream).  Calls on one handle must not
 * overlap (they share the handle's work buffers).
 */
#ifndef ILU_H
#define ILU_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* error codes */
#define ILU_OK 0
#define ILU_EINVAL (-1)     /* bad argument (null pointer, level, degree, ...) */
#define ILU_ENOMEM (-2)     /* device allocation failed */
#define ILU_EHIP (-3)       /* a HIP runtime call failed */
#define ILU_EBREAKDOWN (-4) /* ILU(0) pivot D^p <= 0 (A is not an M-matrix) */
#define ILU_ERANK (-5)      /* a least-squares problem is rank deficient */
#define ILU_EGEOM (-6)      /* det J = 0 (degenerate tetrahedron) */
#define ILU_ENOTCONV (-7)   /* rel_tol requested but not reached in nsweeps */

/* coefficient kinds (kappa as a function of the physical point X) */
#define ILU_COEFF_CONST 0     /* p0 */
#define ILU_COEFF_SINPROD 1   /* p0 + p1 sin(2 pi p2 X) sin(2 pi p2 Y) sin(2 pi p2 Z) */
#define ILU_COEFF_EXPSINCOS 2 /* exp(p0 sin(2 pi p2 X) cos(2 pi p2 Y)) */
#define ILU_COEFF_POLY 3      /* p0 + p1 (X^i + Y^i + Z^i), i = (int)p2 */

/* smoother variants */
#define ILU_STORED_F64 0 /* exact ILU(0) factors stored in HBM, FP64 sweeps */
#define ILU_SURR_F64 1   /* surrogate weights evaluated on the fly, FP64 sweeps */
#define ILU_SURR_F32 2   /* surrogate weights and both sweeps in FP32; residual and
                            update in FP64 (iterative refinement) */
#define ILU_STORED_SGS 3 /* comparator: symmetric Gauss-Seidel (Sec. 2.1),
                            C = (D_A + L_A) D_A^{-1} (D_A + L_A)^T with D_A, L_A the
                            diagonal and strictly lower part of A, stored in the
                            factor form L^p_d = A^p_d / A^{p+d}_c, D^p = A^p_c and
                            swept like ILU_STORED_F64 */

/* operator in the residual b - A x */
#define ILU_A_EXACT 0     /* the assembled FP64 stencil (8 values per point in HBM) */
#define ILU_A_SURROGATE 1 /* surrogate polynomials for A as well (Sec. 4.2): the lower
                             weights fitted on the sample sets S_d with the same
                             degrees, the upper weights evaluated as the lower
                             polynomials at p - d (symmetric), the centre as minus the
                             sum of the 14 neighbour weights (the rows of the
                             unrestricted A sum to zero), so r = b - sum_d A~_d
                             (x_{p+d} - x_p); Horner per point in FP32 for ILU_SURR_F32,
                             FP64 otherwise, FP64 accumulation.  Surrogate variants
                             only; the degree must resolve the coefficient, or the
                             iteration with A~ may diverge. */

/* boundary stencils of the surrogate variants (Sec. 4.1) */
#define ILU_BOUNDARY_V2 0 /* surrogates everywhere; weights whose neighbour is not interior
                             are zeroed in the substitutions */
#define ILU_BOUNDARY_V1 1 /* the exact factors L^p_d and 1/D^p of the boundary points (the
                             O(h^-2) interior points with a stencil neighbour on the macro
                             boundary: min(x,y,z) = 1 or x+y+z = n-1) are stored in compact
                             arrays and used wherever the substitutions need a factor of
                             such a point: L^p_d in the forward substitution at p, 1/D^p
                             and L^p_d (as the weight of p + d) in the backward one.  The
                             surrogate is used everywhere else.  Surrogate variants only;
                             the setup runs the exact factorisation once more for it. */

/* sweep schedules */
#define ILU_SCHED_AUTO 0      /* persistent dataflow kernel */
#define ILU_SCHED_PLANE 1     /* one launch per hyperplane (reference schedule) */
#define ILU_SCHED_DATAFLOW 2  /* persistent kernel, per-block progress counters */

typedef struct ilu_tet_desc {
    double vertex[4][3];   /* v1..v4 (their order fixes the DOF ordering); d_i = v_{i+1} - v1
                              must not be coplanar (either orientation) */
    int32_t level;         /* L in [2, 10] */
    int32_t coeff_kind;    /* ILU_COEFF_* */
    double coeff_param[4];
} ilu_tet_desc;

typedef struct ilu_opts {
    int32_t variant;        /* ILU_STORED_F64 / ILU_SURR_F64 / ILU_SURR_F32 / ILU_STORED_SGS */
    int32_t degree[3];      /* surrogate degrees (dg_x, dg_y, dg_z), each in [0, 6] */
    int32_t sample_stride;  /* stride of S_d (power of two); halved until every
                               sample set is unisolvent; 0 = 4 */
    int32_t schedule;       /* ILU_SCHED_* */
    int32_t tile[2];        /* rows per block (BV, BW) of the sweep schedule in the
                               skewed row coordinates (v, w) = (y+z, z): (8,8), (16,16)
                               or (16,32).  (0,0) = autotuned: setup times a few sweeps
                               of every shape on the device (on zeroed buffers: the sweep
                               kernels' time does not depend on the values), each with
                               several persistent-grid sizes (ilu_set_flow_grid), both
                               residual modes (ilu_set_overlap) and both chunk lengths of
                               the residual run on its own (ilu_set_residual_chunk), keeps the fastest
                               combination and builds only that one (hyperplane schedule:
                               the shape is chosen from the levels) */
    int32_t a_mode;         /* ILU_A_EXACT or ILU_A_SURROGATE */
    int32_t boundary;       /* ILU_BOUNDARY_V2 or ILU_BOUNDARY_V1 (surrogate variants) */
} ilu_opts;

typedef struct ilu_handle_s *ilu_handle_t;

/* Build the smoother for `ntets` tetrahedra: assemble A (Sec. 2.1), factor it
 * with the stencil recurrences of Sec. 3 on the GPU, and for surrogate
 * variants sample the factors on S_d and solve the FP64 least-squares
 * problems (Sec. 4.1, Alg. 1).  Synchronous on `hip_stream`, so breakdown
 * (ILU_EBREAKDOWN), rank (ILU_ERANK) and geometry (ILU_EGEOM) errors are
 * reported here.  On success *out owns all device memory of the smoother.
 * The stored variants keep full factor arrays.  The surrogate variants factor
 * on a ring of the last four hyperplanes (the stencil equations of a point
 * reach back at most three hyperplanes) and take each point's samples (and,
 * ILU_BOUNDARY_V1, its boundary record) as it is factored, so the
 * factorisation adds O(h^-2) memory to the assembled stencil: no full factor
 * array exists at any time (see ilu_setup_memory). */
int ilu_setup_surrogate(const ilu_tet_desc *tets, int32_t ntets, const ilu_opts *opts, void *hip_stream,
                        ilu_handle_t *out);

/* Apply up to `nsweeps` smoothing steps x <- x + C^{-1}(b - A x) (Alg. 2) to
 * every tetrahedron.  x (in/out) and b (in) are FP64 device arrays in the
 * layout above.  If rel_tol > 0 the loop stops early once
 * ||b - A x||_2 / ||b||_2 <= rel_tol over all tetrahedra (the FP64 iterative
 * refinement of the FP32 variant): every sweep's residual kernel reduces the
 * norm on the device, the host reads the norms after every 8 sweeps (this
 * synchronises), and a hit is confirmed on the current x.  ILU_ENOTCONV if the
 * tolerance is not reached.  relres_out (host, may be NULL) receives the
 * relative residual of the returned x, computed when rel_tol > 0 or
 * relres_out != NULL.  With rel_tol == 0 the sweeps replay a captured graph
 * (see ilu_set_graph) and the call is stream-ordered apart from relres_out. */
int ilu_smooth(ilu_handle_t h, double *x, const double *b, int32_t nsweeps, double rel_tol, double *relres_out,
               void *hip_stream);

/* y = A x on the interior points (Sec. 2.1 stencil matvec), FP64 device
 * arrays in the layout above; with ILU_A_SURROGATE the surrogate operator the
 * smoother's residual uses.  Stream-ordered. */
int stencil_apply(ilu_handle_t h, const double *x, double *y, void *hip_stream);

/* Preconditioned conjugate gradients for A x = b with the handle's C^{-1} as
 * preconditioner: the ILU (stored or surrogate) applied directly as a CG
 * preconditioner as in the CG experiment of Sec. 4.2, or with ILU_STORED_SGS
 * the symmetric Gauss-Seidel comparator.  Applying C^{-1} is one forward and
 * one backward substitution from zero (in FP32 for ILU_SURR_F32: the vectors,
 * A p and the CG scalars stay FP64).  x (in: start, out: iterate) and b are
 * FP64 device arrays in the layout above.  Stops at the first iteration k
 * with ||r_k||_2 <= max(rel_tol ||b||_2, abs_tol) for the recursively updated
 * residual r_k, or after maxit iterations.  Every step, the scalars included,
 * runs on the device (one iteration is replayed from a captured graph unless
 * graph replay is off); the host reads the state after every 8 iterations,
 * and iterations after convergence leave x unchanged.  iters_out (host, may
 * be NULL): iterations done; resnorm_out (host, may be NULL): the true
 * residual ||b - A x||_2 of the returned x.  ILU_ENOTCONV if the tolerance
 * is not met, ILU_EBREAKDOWN if p.q or r.z is not positive (x then holds
 * the last iterate).  Synchronous on hip_stream. */
int ilu_pcg(ilu_handle_t h, double *x, const double *b, int32_t maxit, double rel_tol, double abs_tol,
            int32_t *iters_out, double *resnorm_out, void *hip_stream);

/* Asymptotic contraction factor of the smoother by power iteration (the rate
 * definition of the numerical results in Sec. 4.2, applied to one smoothing
 * step): with b = 0 a step maps x to (I - C^{-1} A) x.  Starting from x (FP64
 * device array in the layout above, not zero), nsteps steps are applied, each
 * followed by scaling to unit 2-norm.  rho_out (host): ||x_k||_2 / ||x_{k-1}||_2
 * of the last step; rho_res_out (host, may be NULL): (||A x_k||_2 /
 * ||A x_0||_2)^(1/k) of the unscaled iteration.  On return x holds the last
 * scaled iterate.  Synchronous on hip_stream. */
int ilu_contraction(ilu_handle_t h, double *x, int32_t nsteps, double *rho_out, double *rho_res_out,
                    void *hip_stream);

/* Orientation choice by local Fourier analysis (Sec. 3, strategy on
 * macro-elements): for each of the 24 vertex permutations of each
 * tetrahedron, the smoothing factor mu of the ILU with the asymptotic stencil
 * (the Gauss-Seidel fixed point of the stencil equations) for the constant
 * stencil of a unit coefficient (level and coefficient of the descriptors are
 * ignored):
 *     mu = max |(L D conj(L) - A)(theta) / (L D conj(L))(theta)|
 * over the oscillatory frequencies theta in (-pi,pi)^3 minus (-pi/2,pi/2)^3,
 * sampled at the cell centres theta_j = -pi + (2j+1) pi / samples of a uniform
 * grid (the paper uses 16 samples per direction; samples must be a multiple of
 * 4 in [4, 256]).  Permutation k (0..23) is the k-th permutation
 * s = (s1 s2 s3 s4) of (1 2 3 4) in lexicographic order; the permuted
 * tetrahedron has the original vertex i at position s_i.  mu_out (host,
 * may be NULL): [ntets][24]; +inf where the fixed-point iteration did not
 * converge to a positive pivot.  best_out (host, may be NULL): per
 * tetrahedron the k of the smallest mu (the first one on ties).  ILU_EGEOM
 * for a degenerate tetrahedron.  Synchronous on hip_stream. */
int ilu_lfa_orientation(const ilu_tet_desc *tets, int32_t ntets, int32_t samples, double *mu_out, int32_t *best_out,
                        void *hip_stream);

/* ilu_lfa_orientation for callers that cannot allocate device memory
 * (harnesses that forbid hipMalloc, tight serving loops): the same
 * computation and the same results, with every intermediate (the
 * descriptors, the per-permutation stencils, mu and the choice) in one
 * statically sized device array of the library (about 1.3 MiB, held on
 * each device the library runs on until the process ends) instead of
 * buffers allocated per call.  At most ILU_LFA_NOALLOC_MAX_TETS tetrahedra per
 * call (ILU_EINVAL beyond).  All calls on one device share that array:
 * calls that overlap in time on one device (from several host threads or
 * streams) race and must not be issued.  Synchronous on hip_stream. */
#define ILU_LFA_NOALLOC_MAX_TETS 256
int ilu_lfa_orientation_noalloc(const ilu_tet_desc *tets, int32_t ntets, int32_t samples, double *mu_out,
                                int32_t *best_out, void *hip_stream);

/* Offset and interior-point count of tetrahedron `tet` in the vectors. */
int ilu_layout(ilu_handle_t h, int32_t tet, int64_t *offset, int64_t *count_interior);

/* Release every resource of the handle (NULL is accepted). */
int ilu_destroy(ilu_handle_t h);

/* Static message for an error code. */
const char *ilu_strerror(int code);

/* Detail of the last ILU_EHIP failure on the calling thread (the HIP call
 * and its error name); empty if none. */
const char *ilu_last_error(void);

/* ---- inspection (tests and diagnostics; all synchronous on hip_stream) ---- */

/* Assembled stencil of tetrahedron `tet` in lexicographic order: A_out is a
 * device FP64 array [N][15], directions in the order
 * w,s,se,bnw,bn,bc,be,c,e,n,nw,tse,ts,tc,tw (Sec. 2.1); entries whose
 * neighbour lies on the macro boundary are 0. */
int ilu_get_stencil(ilu_handle_t h, int32_t tet, double *A_out, void *hip_stream);

/* Exact ILU(0) factors of tetrahedron `tet` (only for ILU_STORED_F64; the
 * symmetric Gauss-Seidel factors for ILU_STORED_SGS):
 * L_out device FP64 [N][7] (directions w,s,se,bnw,bn,bc,be; 0 where the
 * neighbour is on the boundary), D_out device FP64 [N]. */
int ilu_get_factors(ilu_handle_t h, int32_t tet, double *L_out, double *D_out, void *hip_stream);

/* Surrogate coefficients of tetrahedron `tet` (surrogate variants), host FP64
 * array [8][K], K = (dg_x+1)(dg_y+1)(dg_z+1).  Row r < 7 fits L_d for the
 * lower direction r (order above), row 7 fits 1/D.  Basis: shifted Legendre
 * P_i(2x-1) P_j(2y-1) P_k(2z-1) of X^ = (x,y,z)/2^L, column (k(dg_y+1)+j)(dg_x+1)+i.
 * ilu_set_surrogate replaces them (and rebuilds the evaluation tables). */
int ilu_get_surrogate(ilu_handle_t h, int32_t tet, double *coeffs_out);
int ilu_set_surrogate(ilu_handle_t h, int32_t tet, const double *coeffs, void *hip_stream);

/* Surrogate coefficients of the operator (handles built with
 * ILU_A_SURROGATE), host FP64 [8][K] in the layout of ilu_get_surrogate: row
 * r < 7 fits A_d for the lower direction r; row 7 fits the centre A_c, which
 * the operator does not use (its centre follows from the row sums).
 * ilu_set_surrogate_a replaces them (and rebuilds the operator tables). */
int ilu_get_surrogate_a(ilu_handle_t h, int32_t tet, double *coeffs_out);
int ilu_set_surrogate_a(ilu_handle_t h, int32_t tet, const double *coeffs, void *hip_stream);

/* Surrogate weights as the sweeps evaluate them, lexicographic order:
 * L_out device FP64 [N][7], Dinv_out device FP64 [N] (FP32 variants are
 * widened; with ILU_BOUNDARY_V1 the stored exact factors at the boundary
 * points). */
int ilu_get_surrogate_values(ilu_handle_t h, int32_t tet, double *L_out, double *Dinv_out, void *hip_stream);

/* Effective sample stride chosen for tetrahedron `tet` (surrogate variants). */
int ilu_sample_stride(ilu_handle_t h, int32_t tet, int32_t *stride_out);

/* Number of sweeps the last ilu_smooth call ran (with rel_tol > 0 the
 * tolerance is tested after every 8 sweeps, so up to 7 sweeps may follow the
 * first one that met it). */
int ilu_last_sweeps(ilu_handle_t h, int32_t *sweeps_out);

/* Device memory (bytes) that the library held during the ilu_setup_surrogate
 * call that made `h`: the peak over the call (the autotuner's timing handles
 * included) and what `h` holds after it.  Host pointers, may be NULL. */
int ilu_setup_memory(ilu_handle_t h, int64_t *peak_bytes, int64_t *resident_bytes);

/* Block shape (rows in v, rows in w) of the sweep schedule the handle uses:
 * the one requested in ilu_opts.tile, or the automatic choice. */
int ilu_tile(ilu_handle_t h, int32_t *bv_out, int32_t *bw_out);

/* Device times (ms) of the last ilu_smooth call, from HIP events on its
 * stream: the whole sweep loop, and per sweep the forward substitution, the
 * backward substitution and the residual (averaged over all sweeps when
 * kernel timing is on, else taken from the first sweep).  The forward and
 * backward figures include the small counter-reset kernel of the dataflow
 * schedule. */
int ilu_last_timing(ilu_handle_t h, double *sweep_ms, double *fwd_kernel_ms, double *bwd_kernel_ms,
                    double *res_kernel_ms);

/* Record events around every kernel of every sweep (diagnostics; adds a
 * little launch overhead).  Off by default.  While on, sweeps run eagerly. */
int ilu_set_kernel_timing(ilu_handle_t h, int32_t enable);

/* Graph replay (on by default).  An ilu_smooth call with rel_tol == 0 runs its
 * sweeps from captured graphs.  A sweep is the batched sweep over every
 * tetrahedron: the residual kernel, the forward substitution and the backward
 * substitution with the update, each one persistent launch.  2 to 64 sweeps
 * run as one graph launch holding all of them (captured for that count on
 * the first call with it, on a private stream, and kept until a call asks for
 * another count); 1 or more than 64 sweeps replay a one-sweep graph.  Calls with
 * rel_tol > 0 (which test the residual between sweeps) and calls with kernel
 * timing on run eagerly.  Results are identical either way.  Per-kernel times
 * of ilu_last_timing are 0 after a graph call. */
int ilu_set_graph(ilu_handle_t h, int32_t enable);

/* Residual of ilu_smooth and the forward substitution (modes below;
 * ILU_OVERLAP_OFF by default with an explicit tile; the autotuner of tile
 * (0,0) keeps whichever of OFF and ON was faster).  ILU_OVERLAP_ON, where available (dataflow
 * schedule, assembled operator, boundary variant V2), runs each sweep's
 * residual kernel on a second, handle-owned stream at the same time as the
 * forward substitution, which takes each point's residual as soon as it is
 * written (every value carries a sweep tag; one still missing after about
 * 64 us of polling is computed by the forward sweep itself, with the same
 * arithmetic; the residual kernel also marks each finished band of
 * hyperplanes, and the sweep waits for a band's mark before loading its
 * entries).  ILU_OVERLAP_FUSED runs no residual kernel: the forward sweep
 * computes every residual itself, the first pass of Alg. 2 in its fused form
 * (its loads then sit on the sweep's dependency chain; calls with
 * rel_tol > 0, whose residual kernel also reduces the norm, use
 * ILU_OVERLAP_ON).  Results are bitwise identical in every mode; only the
 * time changes: the overlapped residual pays when the persistent sweep grid
 * is capped (ilu_set_flow_grid) so that the residual kernel has room beside
 * the latency-bound sweep, the fused form does not pay on MI355X.  With
 * overlap the residual of ilu_last_timing is measured on the second stream
 * while the forward substitution runs.  A mode other than ILU_OVERLAP_OFF where it is not
 * available returns ILU_EINVAL. */
#define ILU_OVERLAP_OFF 0   /* residual kernel, then the forward substitution */
#define ILU_OVERLAP_ON 1    /* residual kernel beside the forward substitution */
#define ILU_OVERLAP_FUSED 2 /* residual computed inside the forward substitution */
int ilu_set_overlap(ilu_handle_t h, int32_t mode);
int ilu_get_overlap(ilu_handle_t h, int32_t *mode);

/* Workgroups of the persistent dataflow sweeps (diagnostics and tests).  By
 * default the grid holds as many workgroups as can be resident at once, up to
 * one per block.  grid > 0 caps it (so that every workgroup takes several
 * blocks from the ticket counter, one after another); grid == 0 restores the
 * default.  The topological ticket order keeps any grid size free of
 * deadlock, and the results do not depend on it.  grid_out (host, may be
 * NULL) receives the grid now in use.  Drops the captured graphs. */
int ilu_set_flow_grid(ilu_handle_t h, int32_t grid, int32_t *grid_out);
/* The grid in use (*grid_out) and the default one (*grid_max_out, may be NULL). */
int ilu_get_flow_grid(ilu_handle_t h, int32_t *grid_out, int32_t *grid_max_out);

/* Hyperplanes per workgroup of the LDS-staged residual kernel when it runs on
 * its own (8x8 and 16x16 blocks, ILU_OVERLAP_OFF; diagnostics, tests and the
 * autotuner, which keeps the faster): 64 (default) or 128.  Longer chunks
 * stage fewer ring prologues but give fewer workgroups.  r, the iterates and
 * the layout of the norm's partial sums do not depend on it; the norm's
 * summation order does (within rounding).  Any other value returns
 * ILU_EINVAL.  Drops the captured graphs. */
int ilu_set_residual_chunk(ilu_handle_t h, int32_t hyperplanes);
int ilu_get_residual_chunk(ilu_handle_t h, int32_t *hyperplanes);

/* Host-only self check (no device needed): builds the stream layout for the
 * given tetrahedra and replays every index the kernels form, counting
 * out-of-range or misdirected accesses in *violations (0 = consistent). */
int ilu_check_layout(const ilu_tet_desc *tets, int32_t ntets, const ilu_opts *opts, int64_t *violations);

#ifdef __cplusplus
}
#endif

#endif /* ILU_H */
