/*
 * mpg.h -- C ABI of the MI355X (gfx950) multipole gravity solver for
 * multi-patch spherical grids, after Wongwathanarat, "A Generalized Solution
 * Method for Parallelized Computation of the Three-dimensional Gravitational
 * Potential on a Multi-patch grid in Spherical Geometry" (arXiv:1903.08475).
 *
 * The library computes, for cell-averaged densities rho on every patch of a
 * grid, the potential Phi at the upper vertex (r_i^+, theta_j^+, phi_k^+) of
 * every cell (Eq. gravpotmult; or at the angular centre on the same outer
 * radius, see mpg_grid.eval_point), in three device steps:
 *   1. moments   B_{i,lm} = sum_g sum_jk rho_{g,i,jk} U_{g,jk,lm}      (Eq. B_CS, Sec. 4.3 step 2)
 *   2. radial sums M_{i,lm} of Eq. M_C (Sec. 4.3 step 4)
 *   3. expansion Phi_{g,i,jk} = sum_lm Q_{g,jk,lm} M_{i,lm}            (Sec. 4.3 step 5)
 * The angular weights U (Eqs. U_C/U_S with the normalisation factors of
 * Eqs. N_CC..N_SC) and prefactors Q (Eqs. Q_C/Q_S) are built once per plan
 * on the device (Sec. 4.3 step 1).
 *
 * Conventions.
 *   - Real moment index: idx(l,0) = l^2, idx(l,m,C) = l^2+2m-1,
 *     idx(l,m,S) = l^2+2m (1 <= m <= l); n_lm = (lmax+1)^2.
 *   - P_l^m carries the Condon-Shortley phase; the prefactor of every
 *     order-m term is 2/delta_m (Eq. del_m).
 *   - A field is rho[n_patches][n_r][n_theta][n_phi], row-major, phi
 *     fastest; a batch of n_fields fields of one plan is n_fields such
 *     arrays back to back.  Phi has the same layout.
 *   - Local patch frames relate to the common frame by x = R^(g) xi with
 *     R^(g) of Eq. rottransmatrix (z-y'-z'' Euler angles).
 *
 * Ownership and execution.  All array arguments of the compute calls are
 * device pointers owned by the caller.  A plan owns its device tables and
 * work space and frees them in mpg_destroy.  Compute calls are enqueued
 * asynchronously on the plan's HIP stream and return at once; errors of
 * the device work surface at the next call or at mpg_sync.  A plan must
 * not be used from two host threads at once.
 *
 * Errors.  Every int-returning call returns MPG_OK (0) or a negative
 * status and never throws; mpg_last_error() gives a message for the last
 * failure of the calling thread.
 */
#ifndef MPG_H
#define MPG_H

#ifdef __cplusplus
extern "C" {
#endif

/* status codes */
#define MPG_OK            0
#define MPG_EINVAL       -1   /* bad argument or grid                      */
#define MPG_ENOMEM       -2   /* device or host allocation failed          */
#define MPG_EDEVICE      -3   /* a HIP call failed                         */
#define MPG_EUNSUPPORTED -4   /* valid request this build does not handle  */

/* arithmetic of the two contractions */
#define MPG_FP64        0     /* FP64 MFMA GEMMs                           */
#define MPG_SPLIT_BF16  1     /* split-BF16 MFMA GEMMs, FP32 accumulation:
                                 six bf16 products per product          */
#define MPG_SPLIT_BF16_TIERED 2 /* as MPG_SPLIT_BF16 with three products
                                 (h*h, h*m, m*h) per product, six on the
                                 moments of degree <= MPG_TIER_LMAX      */
#define MPG_TIER_LMAX   15

/* element types of rho / Phi */
#define MPG_F64 0
#define MPG_F32 1

/* Grid of n_patches geometrically identical patches (Sec. 3).  Every patch
 * spans local colatitudes [theta0, theta0 + n_theta*dtheta] and azimuths
 * [phi0, phi0 + n_phi*dphi]; shells are [r_edges[i], r_edges[i+1]].
 * All pointers are host pointers, read during mpg_plan only. */
typedef struct mpg_grid {
    int n_patches;              /* 1 .. MPG_MAX_PATCHES patches (Sec. 3)     */
    int n_r, n_theta, n_phi;    /* cells per patch                           */
    const double *r_edges;      /* n_r+1, strictly increasing, r_edges[0]>=0 */
    double theta0, phi0;        /* local lower corner                        */
    double dtheta, dphi;        /* local spacing                             */
    const double *euler;        /* n_patches x (alpha, beta, gamma)          */
    const double *overlap_w;    /* cell weights w_jk (see w_per_patch), or NULL */
    double G;                   /* gravitational constant                    */
    int w_per_patch;            /* 0: overlap_w holds n_theta*n_phi weights
                                   shared by every patch; 1: it holds
                                   n_patches*n_theta*n_phi, patch-major      */
    int eval_point;             /* where Phi is evaluated in each cell, on the
                                   outer radius of its shell:
                                   MPG_EVAL_UPPER_VERTEX (0, Eq. gravpotmult)
                                   or MPG_EVAL_ANGULAR_CENTRE (1)            */
} mpg_grid;

#define MPG_EVAL_UPPER_VERTEX 0
#define MPG_EVAL_ANGULAR_CENTRE 1

#define MPG_MAX_PATCHES 16

typedef struct mpg_plan_s *mpg_plan_t;

/* Build a plan: validate the grid, upload its geometry and build the FP64
 * tables U, Q, the overlap weights (Sec. 4.2, w_jk = 1 - alpha_jk/2, when
 * overlap_w is NULL) and the radial recurrence coefficients on the device
 * (Sec. 4.3 step 1), plus their split-BF16 copies for the split forms.
 *   lmax       : truncation degree, 0 <= lmax <= 64
 *   precision  : MPG_FP64, MPG_SPLIT_BF16 or MPG_SPLIT_BF16_TIERED.  The
 *                split forms write each FP32 operand as three bf16 pieces
 *                h + m + l (exact).  MPG_SPLIT_BF16 forms every product
 *                from the six piece products of weight >= 2^-18 of h*h.
 *                MPG_SPLIT_BF16_TIERED keeps those six for the moments of
 *                degree l <= MPG_TIER_LMAX (and the others that share their
 *                64-column wave tile in the moment contraction or their
 *                32-moment K slab in the expansion) and uses the three
 *                products h*h + h*m + m*h (16-bit operands) for the rest:
 *                about 45% less MFMA work at lmax 48.  Its potential stays
 *                within 1e-6 (max-norm relative) of the FP64 result on the
 *                test workloads.  The moments B and M that mpg_moments
 *                returns are formed with six products on every column in
 *                both split forms (within 1e-6 of max|B|); the tiered
 *                three-product moments only feed the expansion inside
 *                mpg_potential.
 *   max_fields : largest n_fields later passed to the compute calls (>= 1);
 *                sizes the work space
 *   stream     : hipStream_t on which the plan runs (NULL: default stream)
 * Two patches whose rotations differ by pi about the local polar axis
 * (R^(1) = diag(-1,-1,1) R^(0), as for Yin and Yang) use the parity fold
 * (U_Yang = (-1)^m U_Yin, Sec. 4.2): one table and contractions over
 * rho_Yin +- rho_Yang.  Every other set of patches (any n_patches, any
 * Euler angles; Sec. 3) takes the general path: tables of every patch and
 * contractions over all patches' cells at once.
 * Overlap weights: NULL gives w = 1 for one patch, and the closed-form
 * Yin-Yang weights for two patches related by the Yin<->Yang map
 * (R^(0)T R^(1) = P of Eq. caryytransform) with extents symmetric about
 * the patch centre; other grids must pass overlap_w (else
 * MPG_EUNSUPPORTED).  Blocks until the tables are built.
 * Errors: MPG_EINVAL, MPG_ENOMEM, MPG_EDEVICE, MPG_EUNSUPPORTED. */
int mpg_plan(const mpg_grid *grid, int lmax, int precision, int max_fields,
             void *stream, mpg_plan_t *out);

/* methods of mpg_plan_method */
#define MPG_METHOD_GLOBAL    0  /* the paper's method (mpg_plan): one moment set
                                   in the common frame for all patches       */
#define MPG_METHOD_PER_PATCH 1  /* the comparison method the paper sets its
                                   own against (Sec. 1, Sec. 4.3): moments of
                                   every patch in its own frame, radial sums
                                   per patch, and an expansion that adds the
                                   potentials of every patch's source        */
#define MPG_METHOD_SEPARABLE 2  /* the paper's method with each angular
                                   contraction factored over the patch's
                                   (theta, phi) cell grid: see below         */

/* As mpg_plan, with the method chosen.  The per-patch method gives the same
 * potential up to rounding (the degree-l part of each patch's expansion
 * does not depend on the frame) at about twice the moment work and four
 * times the expansion work for two patches; it is here for the comparison.
 * It uses one table U for every patch (so per-patch weights must agree),
 * mpg_moments returns B and M per patch ([n_fields][n_patches][n_r][n_lm],
 * each in the patch's own frame), and mpg_potential_batch rejects it
 * (MPG_EUNSUPPORTED).
 *
 * MPG_METHOD_SEPARABLE computes the same B, M and Phi as the paper's
 * method (Eqs. B_CS, M_C, gravpotmult) in fewer operations.  In each
 * patch's own frame the weights of its cell (j, k) factor over theta and phi
 * (the single-grid sums of Eqs. a_ci^lm/a_si^lm): the local moments are a
 * phi transform of every (field, patch, shell, theta row) row followed by a
 * theta contraction per order u, A^(lu) = sum_j s_lu T_j^(lu) sum_k w_jk
 * rho_jk {C_k^u, S_k^u}; the N factors of Eqs. U_C/U_S rotate them into
 * the common frame degree by degree and the patches' sums are added.  The
 * expansion rotates M into each patch's frame and runs the two transforms
 * backwards (the same factors write the harmonics of Eqs. Q_C/Q_S in local
 * ones).  On a phi grid symmetric about 0 with an even cell count the phi
 * transforms fold cell k with its mirror cell n_phi - 1 - k.  Operations
 * per shell and patch: about n_theta n_phi (2 lmax + 1) (halved by the
 * mirror fold) against n_theta n_phi (lmax + 1)^2 for the dense
 * contraction (under the parity fold, per patch pair).  Precision
 * MPG_FP64, or MPG_SPLIT_BF16: the two phi transforms then run as six bf16
 * piece products with FP32 accumulation (at most 2 (n_phi / 2) terms
 * each) into FP64 work arrays, with the order-0 column, theta
 * contractions, rotations and scans in FP64 (about 1e-8 relative to FP64);
 * MPG_SPLIT_BF16_TIERED gives MPG_EUNSUPPORTED.  Any patches and Euler
 * angles.  mpg_potential_static, mpg_potential_batch, mpg_autotune and
 * mpg_set_tuning reject such plans (MPG_EUNSUPPORTED); mpg_moments,
 * mpg_potential, mpg_tables and stage timing take them (stages: phi
 * transform of the moments; theta contractions and rotations of moments
 * and expansion; radial scans; phi transform of the expansion).  The plan holds two extra FP64 work arrays:
 * (lmax + 1 and lmax, each rounded up to 16) x max_fields x n_patches x
 * n_r x n_theta values, and max_fields x n_patches x n_r x (lmax + 1)^2.
 * Errors: as mpg_plan, MPG_EINVAL for an unknown method. */
int mpg_plan_method(const mpg_grid *grid, int lmax, int precision, int max_fields,
                    int method, void *stream, mpg_plan_t *out);

/* Moments only (Eq. B_CS and Eq. M_C).
 *   rho   : device, n_fields fields of rho_dtype
 *   B, M  : device FP64 [n_fields][n_r][n_lm] in the real index, or NULL
 * The split forms contract with six bf16 products on every column here
 * (the tiered form included).  Any number of (field, shell) rows.
 * Errors: MPG_EINVAL (n_fields out of [1, max_fields], bad dtype, null
 * rho), MPG_EDEVICE. */
int mpg_moments(mpg_plan_t plan, int n_fields, const void *rho, int rho_dtype,
                double *B, double *M);

/* The whole solve (Sec. 4.3 steps 2-5) for n_fields fields of one plan.
 *   rho : device input, rho_dtype;  phi : device output, phi_dtype
 * Errors: as mpg_moments. */
int mpg_potential(mpg_plan_t plan, int n_fields, const void *rho, int rho_dtype,
                  void *phi, int phi_dtype);

/* The whole solve as mpg_potential, allocating nothing: for callers that
 * cannot allocate device memory (code under HIP graph capture, serving
 * loops, harnesses that forbid hipMalloc).  The work arrays of the call
 * (K-split partial moments, B, M and, in the split forms, the bf16 pieces
 * of the input and of M) live in one static device array of
 * MPG_STATIC_WORKSPACE_MB MiB per GPU, part of the library's code object
 * and held until the process ends, instead of the plan's work space; the
 * plan supplies only its tables.  The plan's K split choice is reduced
 * until the call's arrays fit; a call that does not fit even with one
 * split fails with MPG_EINVAL and a message stating the size it needs.
 * Nothing in the array needs clearing between calls: every entry a call
 * reads it writes first.  Calls that overlap on one GPU (on different
 * streams or host threads) race on the array and must be serialized by the
 * caller.  The plan's device must be current.  No stage timing.
 * Arguments, layout and errors as mpg_potential. */
#define MPG_STATIC_WORKSPACE_MB 64
int mpg_potential_static(mpg_plan_t plan, int n_fields, const void *rho, int rho_dtype,
                         void *phi, int phi_dtype);

/* Solve n independent fields with different plans (grid sizes and lmax)
 * together.  Split forms: one persistent kernel (one block per CU) takes
 * the tiles of every stage of every field (input split, moments, radial
 * scans, expansion) from one queue, whose order (fixed on the host by a
 * list-scheduling simulation) puts every tile after the tiles of its
 * field's previous stage; a tile waits on device counters until that stage
 * has finished (a bounded wait: past about 4 s it gives up, every block
 * drains, and mpg_batch_field_times reports it), so small fields complete
 * early.  Each field takes its plan's block shapes of both contractions
 * and its scan chunks (autotuned or set); its moment contraction is split
 * along K only as far as needed for tiles of at most about 0.5 ms (a single
 * solve's autotuned K split is not used: the other fields fill the chip;
 * mpg_batch_choices reports the split).  FP64: one persistent work-queue
 * kernel per stage (moments, radial scans, expansion), each holding the
 * tiles of every field, longest first, with each plan's K split and scan
 * chunks.  The launches are captured once in
 * a hipGraph (per set of plans and dtype) and replayed; a later
 * mpg_autotune or mpg_set_tuning of one of the plans makes the next call
 * capture afresh.  rho[f] and phi[f] are device
 * pointers of field f, each holding exactly one field of plans[f]'s grid
 * (the library cannot check their sizes), of element type dtype.  The plans must be distinct and
 * share precision; the work runs on plans[0]'s stream.  Not for concurrent
 * use from several host threads with the same plans.
 * Errors: MPG_EINVAL, MPG_ENOMEM, MPG_EDEVICE, MPG_EUNSUPPORTED (a plan of
 * the per-patch method). */
int mpg_potential_batch(int n, const mpg_plan_t *plans, const void *const *rho,
                        void *const *phi, int dtype);

/* Completion times of the fields of the last mpg_potential_batch call with
 * these plans (same list and order) and dtype, for measuring per-field
 * latency inside one batched solve: ms[f] (host, n entries) receives the
 * time from the start of the batched solve on the device to the moment the
 * last expansion tile of field f finished, read from the device wall
 * clock.  Waits for plans[0]'s stream.
 * Errors: MPG_EINVAL (bad arguments, or no batched solve of these plans
 * and dtype), MPG_EDEVICE (also when a stage wait of that solve gave up:
 * its results are then incomplete). */
int mpg_batch_field_times(int n, const mpg_plan_t *plans, int dtype, double *ms);

/* The choices each field takes in a batched solve (mpg_potential_batch)
 * of these plans in this dtype: per field f, splitk[f] the K split of its
 * moment contraction, chunks[f] its scan's shell chunks per column, and
 * gemm1_rows[f], gemm2_rows[f] the block shapes of its contractions (as in
 * mpg_set_tuning; gemm2_rows 1 for the FP64 form).  Each pointer is a host array of n
 * entries, or NULL.  A single solve with these choices set
 * (mpg_set_tuning) gives the batched field's results bit for bit.
 * Errors: MPG_EINVAL (bad arguments). */
int mpg_batch_choices(int n, const mpg_plan_t *plans, int dtype, int *splitk, int *chunks,
                      int *gemm1_rows, int *gemm2_rows);

/* Autotune the plan for n_fields fields on the given device input, and keep
 * the choices for later calls:
 *  - the moment contraction's block shape and K split, every pair timed
 *    together with the radial scan that reduces the partial sums.  Shapes:
 *    split forms 128 rows x 256 columns (gemm1_rows = 1, the default) or
 *    256 x 128 (gemm1_rows = 2); FP64 tiles of 128 x 128 (1, the default)
 *    or 64 x 64 (2).  K splits: the default choice first, then 1, 2, 3, 4
 *    and the powers of two beyond, as far as the work space allows (at
 *    least four splits when their partial sums fit in 2 GiB, up to 32
 *    while they fit in 512 MiB).  Each shape keeps its default split
 *    unless another is at least 1% faster, and single-plan calls keep the
 *    default shape unless the other is at least 1% faster;
 *  - the radial scan's shell chunks per column: 4, 8, 12 or 16;
 *  - split forms: the expansion's block shape, 128 rows x 256 angular cells
 *    (gemm2_rows = 1, the default) or 256 x 128 (gemm2_rows = 2).  Its
 *    timing writes a temporary output of one call's size, allocated and
 *    freed here; if it cannot be allocated, the shape is left as it is.
 * Candidates are timed in rounds that launch each of them once (three
 * rounds after a warm-up round), and each keeps its fastest time, so that
 * clock changes during the tuning weigh on all alike.  The expansion's two
 * shapes, and for batched calls (mpg_potential_batch) the moment
 * contraction's two shapes without a K split, are ranked by chip work: the
 * time of one block (a shape's time over its waves of one block per CU)
 * times its blocks, over the CUs; that is its time when its blocks fill
 * whole waves, and otherwise leaves out the CUs a partial wave leaves
 * idle, which the other fields of a batch use.  The one with at least 1%
 * less chip work is kept; otherwise the one with fewer blocks (padding
 * included), and the default when those are equal too.  Batched calls take
 * the scan chunks, the expansion shape and that moment shape, and split K
 * their own way.
 * Blocks until done; overwrites the plan's work space.  splitk, chunks,
 * gemm1_rows and gemm2_rows (each may be NULL) receive the single-plan
 * choices (gemm2_rows: 1 for the FP64 form).  On an error the plan keeps
 * its previous choices.
 * Errors: as mpg_moments. */
int mpg_autotune(mpg_plan_t plan, int n_fields, const void *rho, int rho_dtype,
                 int *splitk, int *chunks, int *gemm1_rows, int *gemm2_rows);

/* Set the choices mpg_autotune makes, e.g. ones it made earlier for the same
 * grid and lmax: the K split of the moment contraction (at most the plan's
 * work space allows), the radial scan's shell chunks per column (1..16),
 * and the contractions' block shapes: gemm1_rows and gemm2_rows 1 (the
 * default) or 2, in the split forms 128 rows x 256 columns or angular
 * cells (1) or 256 x 128 (2), for the FP64 moment contraction tiles of
 * 128 x 128 (1) or 64 x 64 (2) (the FP64 expansion has one shape).  A
 * value <= 0 leaves that choice as it is; a moment shape set here holds
 * for batched calls too.  Results do not depend on the shapes; they may
 * differ in rounding with the K split and the chunks.
 * Errors: MPG_EINVAL (NULL plan, a value out of range; nothing is changed). */
int mpg_set_tuning(mpg_plan_t plan, int splitk, int chunks, int gemm1_rows, int gemm2_rows);

/* Copy the plan's FP64 tables to device buffers, in the real index:
 *   U : [n_patches][n_theta*n_phi][n_lm]   (Eqs. U_C/U_S), or NULL
 *   Q : [n_patches][n_theta*n_phi][n_lm]   (Eqs. Q_C/Q_S), or NULL
 *   w : [n_patches][n_theta*n_phi] overlap weights, or NULL
 * For checking the table build; not needed for solving. */
int mpg_tables(mpg_plan_t plan, double *U, double *Q, double *w);

/* Sizes of a plan: n_lm and the element count of one field. */
int mpg_plan_info(mpg_plan_t plan, int *n_lm, long long *field_elems);

/* Per-stage device timing, for measurement.  With enable != 0 every later
 * compute call of the plan records HIP events on the plan's stream around
 * its stages: 0 = input split (split-BF16 only: rho_Yin +- rho_Yang as bf16
 * pieces), 1 = moment contraction, 2 = radial scan, 3 = expansion (the
 * separable method: 0 = phi transform of the moments, 1 = theta
 * contractions and rotations of both steps, 3 = phi transform of the
 * expansion; each solve counts two launches of stage 1).
 * mpg_stage_times waits for the stream and returns the summed milliseconds
 * and launch counts per stage since the last reset (reset != 0 clears them
 * after reading); ms and launches (4 entries each) may be NULL.
 * Errors: MPG_EINVAL, MPG_ENOMEM, MPG_EDEVICE. */
int mpg_timing(mpg_plan_t plan, int enable);
int mpg_stage_times(mpg_plan_t plan, double ms[4], long long launches[4], int reset);

/* Wait for the plan's stream; reports device errors. */
int mpg_sync(mpg_plan_t plan);

/* Free the plan and its device memory (waits for its stream first). */
void mpg_destroy(mpg_plan_t plan);

/* Message of the calling thread's last failure ("" if none). */
const char *mpg_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
