/*
 * laueot.h -- C ABI of the MI355X (gfx950) LaueOT hot-path library.
 *
 * The library implements the data-parallel hot path of Laue indexing with
 * optimal transport (Kacprzak et al., "Laue Indexing with Optimal Transport"):
 *   - the forward model (Sec. 3.2-3.3: Eqs. ray_mnt, s_mnt, wavelength,
 *     model_spot_cut),
 *   - the assignment cost and the entropic-OT E-step with an outlier row and
 *     column (Sec. 4: Eqs. likelihood, update_L, elbo, estep_obj;
 *     Alg. BalancedOT), run as a streamed log-domain Sinkhorn that never
 *     materialises the detected x model matrix,
 *   - the per-grain M-step (Sec. 4.4, Eq. mstep_obj) as a weighted
 *     Gauss-Newton step over rotation and position with FP64 6x6 solves,
 *   - the multigrain EM driver (Alg. LaueOT) and a simulator of detected spots
 *     (Sec. 3.3.1, Eq. spot_noisy) for synthetic inputs.
 *
 * Conventions (apply to every entry point):
 *   - Units: millimetres, Angstrom, radians; costs and temperatures in mm^2.
 *     The beam is e = (1,0,0).
 *   - "device" pointers are HIP device memory owned by the caller; "host"
 *     pointers are ordinary host memory owned by the caller.  The library
 *     never allocates device memory: entry points that need scratch take a
 *     caller-allocated device workspace (ws, ws_bytes) whose minimum size the
 *     matching *_workspace_size query returns.  Workspaces must be 256-byte
 *     aligned and must not be shared by calls that may overlap.
 *   - stream is a hipStream_t passed as void*.  NULL means the default
 *     stream.  Unless stated otherwise, calls enqueue work and return; calls
 *     documented as "synchronous" wait for their stream before returning.
 *   - Return value: LAUE_OK (0) on success, a negative LAUE_E* code on error
 *     (nothing was enqueued, outputs are unspecified), or a positive warning
 *     (results valid).  laue_last_error() gives the message of the last
 *     failure on the calling thread.
 *   - Arrays are structure-of-arrays.  Detected and model spots are sorted by
 *     block b = t * n_det + d (rotation t, detector d) and described by CSR
 *     block offsets; model spots are additionally sorted by grain, then plane,
 *     inside each block (the order laue_forward_enumerate produces).
 *   - Precision: geometry and Sinkhorn arithmetic in FP32; the 6x6 normal
 *     equations, per-grain reductions, marginal errors, bin potentials and
 *     likelihood accumulations in FP64.
 */
#ifndef LAUEOT_H
#define LAUEOT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define LAUE_OK 0
#define LAUE_ENOCONV 1          /* warning: Sinkhorn stopped at its iteration cap */
#define LAUE_EINVAL (-1)        /* invalid argument (null pointer, bad size, NaN) */
#define LAUE_EINFEASIBLE (-2)   /* T_a = T_b + |I| - |J| < 0 */
#define LAUE_ECAPACITY (-3)     /* output capacity too small; required size reported */
#define LAUE_EDEVICE (-4)       /* a HIP runtime call failed */
#define LAUE_EWORKSPACE (-5)    /* workspace missing, too small or misaligned */

#define LAUE_MAX_DET 4
#define LAUE_MAX_ROT 360

/* Version of this ABI (major * 10000 + minor * 100 + patch). */
int laue_version(void);

/* Message of the last error on the calling thread ("" if none).  The string
 * stays valid until the next library call on that thread. */
const char *laue_last_error(void);

/* ---- problem description ---------------------------------------------- */

/* A flat square detector (Sec. 3.3.1: centre gamma, normal nu, side l).
 * axis1, axis2: in-plane unit axes; detector-local coordinates of a point P
 * on the detector are (axis1.(P - center), axis2.(P - center)). */
typedef struct laue_detector {
    double center[3];
    double normal[3];
    double axis1[3];
    double axis2[3];
    double half_size;           /* l / 2 */
} laue_detector;

/* Scan, detectors and band.  Sample rotation t is Gamma_t = R_z(omega0 +
 * t * domega) about (0,0,1) (Sec. 3.3); band [lambda_min, lambda_max]
 * (Eq. model_spot_cut). */
typedef struct laue_geometry {
    int32_t n_rot;              /* T, 1 .. LAUE_MAX_ROT */
    int32_t n_det;              /* 1 .. LAUE_MAX_DET */
    double omega0, domega;
    double lambda_min, lambda_max;
    laue_detector det[LAUE_MAX_DET];
} laue_geometry;

/* Miller-plane set {(w_m, d_m)} (Sec. 3.3), device arrays.
 * w: [n][3] unit normals in the crystal frame; d: [n] spacings (A);
 * harmonic_prev: [n] index of the parallel plane of next lower order, or -1
 * (used to merge harmonics, which produce identical spots). */
typedef struct laue_planes {
    int32_t n;
    const float *w;
    const float *d;
    const int32_t *harmonic_prev;
} laue_planes;

/* Grains G_n = (R_n, x_n) (Sec. 3.3), device arrays, FP64.
 * q: [n][4] unit quaternions (w,x,y,z); x: [n][3] positions (mm). */
typedef struct laue_grains {
    int32_t n;
    double *q;
    double *x;
} laue_grains;

/* Detected spots {p_i, t_i} (Sec. 3.3.1), device arrays sorted by block.
 * p1, p2: [n] detector-local coordinates (mm).  block_off: HOST [n_blocks+1]
 * CSR offsets (n_blocks = n_rot * n_det). */
typedef struct laue_obs_spots {
    int64_t n;
    const float *p1;
    const float *p2;
    const int64_t *block_off;
} laue_obs_spots;

/* Model spots (Eq. model_spot_cut), device SoA arrays of length n sorted by
 * block, then grain, then plane.  block_off: HOST [n_blocks+1].
 * Geometry arrays (filled by laue_forward_enumerate / laue_forward_eval):
 *   s1, s2     detector-local spot position (mm);
 *   vn, v1, v2 ray vector s - Gamma_t x_n in the detector frame (normal,
 *              axis1, axis2) (mm);
 *   lam        Bragg wavelength (A) (may be NULL);
 *   flags      bit0: within 1e-6 A of a band edge; bit1: within 1e-4 mm of a
 *              detector edge (may be NULL). */
typedef struct laue_model_spots {
    int64_t n;
    int32_t *plane;
    int32_t *grain;
    int32_t *block;
    float *s1, *s2;
    float *vn, *v1, *v2;
    float *lam;
    uint8_t *flags;
    int64_t *block_off;
} laue_model_spots;

/* ---- host helper ------------------------------------------------------- */

/* Cubic plane list (Sec. 3.1: d = a / sqrt(h^2+k^2+l^2)).  All signed
 * (h,k,l) != 0 with h^2+k^2+l^2 <= n_max surviving the extinction rule of
 * centering 'P' (none), 'I' (h+k+l even) or 'F' (all even or all odd),
 * ordered by (N, h, k, l).  HOST arrays; pass NULL arrays to query *n_planes.
 * hkl [n][3], w [n][3] (unit normal), d [n], harmonic_prev [n]. */
int laue_planes_cubic(double a, char centering, int n_max, int32_t *n_planes,
                      int32_t *hkl, float *w, float *d, int32_t *harmonic_prev);

/* ---- forward model ------------------------------------------------------ */

/* Workspace for laue_forward_enumerate / laue_simulate. */
size_t laue_forward_workspace_size(const laue_geometry *geom, int32_t n_planes, int32_t n_grains);

/* Visible reflections of grains (Eq. model_spot_cut), in block, grain, plane
 * order.  merge_harmonics = 0: every plane in band and on a detector (the
 * literal set); 1: of parallel planes giving the same spot keep only the
 * lowest order.  out->n is the capacity on entry; on return *n_out (HOST) is
 * the number found and out->block_off is filled.  If *n_out > capacity the
 * call returns LAUE_ECAPACITY and writes no spot.  Synchronous. */
int laue_forward_enumerate(const laue_geometry *geom, const laue_planes *planes,
                           const laue_grains *grains, int merge_harmonics,
                           laue_model_spots *out, int64_t *n_out,
                           void *ws, size_t ws_bytes, void *stream);

/* The write half of laue_forward_enumerate (Eq. model_spot_cut), for a call
 * that follows one of laue_forward_enumerate on the same workspace (typically
 * the capacity query, out->n = 0, that returned LAUE_ECAPACITY): the counts,
 * offsets and kept-plane bits that call left in ws are written out without
 * counting again.  geom, planes, grains (the same arrays) and merge_harmonics
 * must be those of that call; the library checks the sizes, the geometry and
 * the array pointers (LAUE_EINVAL on a mismatch, or when the workspace holds
 * no count), but not their contents: neither the grain arrays nor the
 * workspace may change in between (no other call on ws).  Capacity,
 * *n_out, out->block_off and the result are as for laue_forward_enumerate.
 * Synchronous. */
int laue_forward_enumerate_counted(const laue_geometry *geom, const laue_planes *planes,
                                   const laue_grains *grains, int merge_harmonics,
                                   laue_model_spots *out, int64_t *n_out,
                                   void *ws, size_t ws_bytes, void *stream);

/* Forward model on a frozen list (Sec. 4.2: the model-spot set is fixed at
 * the prototypes): recomputes s1, s2, vn, v1, v2 (and lam) of every spot of
 * `spots` from its (plane, grain, block) at the given grains; no filtering. */
int laue_forward_eval(const laue_geometry *geom, const laue_planes *planes,
                      const laue_grains *grains, laue_model_spots *spots,
                      void *ws, size_t ws_bytes, void *stream);

/* Workspace for laue_simulate: n_true_max bounds the harmonic-merged visible
 * spots of the truth (laue_forward_enumerate with capacity 0 returns it),
 * n_obs_max the output capacity. */
size_t laue_simulate_workspace_size(const laue_geometry *geom, int32_t n_planes, int32_t n_grains,
                                    int64_t n_true_max, int64_t n_obs_max);

/* Synthetic detected spots (Sec. 3.3.1, Eq. spot_noisy): the harmonic-merged
 * model spots of `truth`, each ray perturbed by an isotropic Gaussian of
 * angular sigma sigma_mm / distance and renormalised, re-intersected with its
 * detector (spots leaving it are dropped); plus, per block, floor(frac *
 * n_true + 0.5) outliers uniform on the detector; ordered per block by a
 * 64-bit random key (ties: true spots first, then by index).  Random numbers:
 * Philox4x32-10 keyed by (seed low word, seed high word) with counters
 * (n, t, m + 65536 d, 1) for ray noise, (k, t, 65536 d, 2) for outlier k,
 * (n, t, m + 65536 d, 3) / (k, t, 65536 d, 4) for order keys; uniforms
 * (x + 0.5) / 2^32, Gaussians by Box-Muller.  The simulator runs in FP64.
 * Outputs (device, capacity = *n_out on entry): p1, p2, grain (-1 outlier),
 * plane (-1 outlier); block_off (HOST [n_blocks+1]).  Returns LAUE_ECAPACITY
 * with the required *n_out if the capacity is too small (no spot written),
 * or with *n_out = -(visible spots) if n_true_max is too small.
 * Synchronous. */
int laue_simulate(const laue_geometry *geom, const laue_planes *planes,
                  const laue_grains *truth, double sigma_mm, double distance,
                  double outlier_frac, uint64_t seed, int64_t n_true_max,
                  float *p1, float *p2, int32_t *grain, int32_t *plane,
                  int64_t *block_off, int64_t *n_out,
                  void *ws, size_t ws_bytes, void *stream);

/* ---- E-step: streamed log-domain Sinkhorn -------------------------------- */

/* Costs and marginals (Sec. 4, Eq. update_L; Sec. 4.3).  Pair cost
 * c_ij = D^2 ||rhat_ij - r_j||^2 (mm^2) for a detected and a model spot of
 * the same block (rhat: unit vector from the grain centre to the detected
 * spot; r: model ray), i.e. the likelihood L_ij = sigma^-2 rhat^T r up to a
 * constant with sigma = sigma_mm / D.  Bins: c_out for a detected spot in the
 * outlier column, c_unm for a model spot in the unmatched row, c_sink for
 * Q_00.  Marginals: 1 per spot, T_b for row 0 and T_a = T_b + |I| - |J| for
 * column 0. */
typedef struct laue_ot_params {
    double eps;                 /* entropic temperature (mm^2) */
    double distance;            /* D (mm) */
    double c_out, c_unm, c_sink;
    double t_b;
    double tol;                 /* stop when max relative row-marginal error <= tol, or
                                 * when it is <= 4 tol and has not fallen by 1% over
                                 * 64 iterations (the rounding floor of FP32
                                 * potentials); both count as converged */
    int32_t n_max;              /* iteration cap (>= 1) */
    int32_t chunk;              /* iterations between host polls (0: 16; in an EM, sized
                                 * per temperature stage) */
    /* sparse assignment (Sec. 5.2): 0 dense; 8, 16 or 32 = every detected
     * spot keeps only its rho nearest model spots of its block by the chord
     * cost (ties to the lower index), the plan being null elsewhere (the bins
     * stay).  The sets are chosen afresh before every Sinkhorn (and before a
     * lone M-step) from that call's model-spot columns.  The workspace then
     * comes from laue_sparse_workspace_size. */
    int32_t rho;
    /* outlier treatment: 0 = the outlier row and column of Sec. 4.3 (bins
     * c_out, c_unm, c_sink and mass T_b); 1 = unbalanced OT (App. C,
     * Problem B): no bins (c_out, c_unm, c_sink and t_b are ignored; the bin
     * potentials come back as -inf), the row and column marginals relaxed by
     * KL penalties of strengths kappa (detected spots) and lam (model spots),
     * in mm^2 like eps (a strength k in log-likelihood units is
     * k * 2 sigma_mm^2).  Rows update as f <- tau_r (f - eps ln S_row),
     * columns as g <- tau_c (g - eps ln S_col), with tau_r = kappa / (kappa +
     * eps), tau_c = lam / (lam + eps) and S the previous state's plan sums; a
     * row or column with no entry gets potential 0.  Stop when the largest
     * change an update of the iteration makes to a row or column marginal of
     * the plan, S |exp(du / eps) - 1| (S its mass before the update, du its
     * potential change), is <= tol (or, as above, within 4 tol and stalled
     * for 64 iterations).
     * 2 = partial OT (App. C, Problem A): no bins either; plans with row and
     * column sums <= 1 and total mass m = m_frac * sum_b min(|I_b|, |J_b|)
     * (the most the block plans can carry), the KL projection of the Gibbs
     * kernel exp(-c/eps) by Dykstra's projections (Alg. PartialOT), in
     * potential form: f = min(0, -eps LSE_j (g_j + H - c_ij)/eps), g likewise
     * over the column, then H += eps ln(m / M) with M the mass after the
     * column step.  Every solve starts from the Gibbs kernel (the given f and
     * g are not read); on return H is folded into f, so that
     * Q = exp((f + g - c)/eps).  Stop when the largest change between
     * consecutive iterations of a row mass (of the plan entering the row
     * step) or a column mass (of the plan entering the column step) is <= tol
     * (or within 4 tol and stalled for 64 iterations). */
    int32_t outlier_model;
    double kappa, lam;
    double m_frac;              /* partial OT: fraction of the mass transported, (0, 1] */
} laue_ot_params;

/* The outlier row and column of Sec. 7 for a spot noise of sigma_mm at
 * detector distance D (host helper, writes every field of *out):
 * c_out = 2 D^2 (1 - cos(3 sigma_mm / D)) (the likelihood of an angular miss
 * of 3 sigma), c_unm = 0 (the null angle), c_sink = c_out,
 * t_b = ceil(0.4 n_model) (at most 40% of the model spots unmatched),
 * eps = 2 sigma_mm^2 (the paper's temperature 1, plain EM), tol = 1e-5,
 * n_max = 2000, chunk = 0, rho = 0 (dense), outlier_model = 0, kappa = lam =
 * m_frac = 0.  LAUE_EINVAL for a non-positive sigma_mm or distance or a
 * negative n_model. */
int laue_ot_defaults(double sigma_mm, double distance, int64_t n_model, laue_ot_params *out);

/* Dual potentials: Q_ij = exp((f_i + g_j - c_ij) / eps).  f [n_obs], g
 * [n_model] device FP32 (in: warm start, out: result); f0, g0 host FP64. */
typedef struct laue_potentials {
    float *f;
    float *g;
    double f0, g0;
} laue_potentials;

typedef struct laue_ot_stats {
    int32_t n_iter;             /* completed row+column iterations */
    int32_t converged;
    double err;                 /* the stopping test's value at the end: max relative
                                 * row-marginal error (outlier_model 0), largest
                                 * marginal change of an update (outlier_model 1),
                                 * largest plan-mass change between iterations (2) */
} laue_ot_stats;

size_t laue_sinkhorn_workspace_size(const laue_geometry *geom, int64_t n_obs, int64_t n_model,
                                    int32_t n_grains);

/* Sinkhorn iterations (Alg. BalancedOT in the log domain) from the given
 * potentials: row half (all f_i and f_0 from g, g0), then column half (all
 * g_j and g_0 from the new f, f0), until the max relative row-marginal error
 * after a column half is <= tol or n_max iterations.  With
 * par->outlier_model = 1 or 2 the iterations are those of Alg. UnbalancedOT
 * or Alg. PartialOT instead (see laue_ot_params; f0, g0 are then not read and
 * come back as -inf).  Uses the model spots' s1, s2, vn, v1, v2.  Synchronous.  Returns
 * LAUE_ENOCONV at the cap. */
int laue_sinkhorn(const laue_geometry *geom, const laue_obs_spots *obs,
                  const laue_model_spots *model, const laue_ot_params *par,
                  laue_potentials *pot, laue_ot_stats *stats,
                  void *ws, size_t ws_bytes, void *stream);

/* laue_sinkhorn for callers that cannot allocate device memory (code under
 * HIP graph capture elsewhere in their program, serving loops, harnesses that
 * forbid hipMalloc): the same iterations, kernels and results, bit for bit,
 * with no workspace argument.  Its scratch is a fixed device array of the
 * library, laue_sinkhorn_noalloc_capacity() = 64 MiB per GPU, held by each GPU
 * the call runs on from the first call until the process ends; the call
 * allocates no device memory and creates no HIP event, stream or graph
 * (direct launches, one spot per lane, no timing).  A problem whose
 * workspace (laue_sinkhorn_workspace_size, or laue_sparse_workspace_size for
 * rho > 0) exceeds the capacity returns LAUE_ECAPACITY and enqueues nothing.
 * Every call on a GPU shares that GPU's scratch, which keeps the last call's
 * contents (every call rewrites what it reads): calls that overlap on one GPU
 * (several host threads or streams) race and must be serialised by the
 * caller.  Synchronous; LAUE_ENOCONV at the cap. */
size_t laue_sinkhorn_noalloc_capacity(void);
int laue_sinkhorn_noalloc(const laue_geometry *geom, const laue_obs_spots *obs,
                          const laue_model_spots *model, const laue_ot_params *par,
                          laue_potentials *pot, laue_ot_stats *stats, void *stream);

/* FP64 summaries of the plan of (pot, par->eps) and its bins (Eqs. elbo,
 * estep_obj): mass (every entry, bins included), cost_inlier = <c, Q> over
 * the detected x model entries, cost_total with the bin entries at c_out,
 * c_unm, c_sink, entropy = -sum Q ln Q, and sem_objective = kappa * mass -
 * cost_total / (2 sigma^2) + eps / (2 sigma^2) * entropy with
 * kappa = (D / sigma)^2, the paper's log-likelihood objective in its units
 * (outlier row and column only; NaN for unbalanced and partial OT, whose
 * plans have no bins).  Under the sparse assignment only kept entries count.
 * Host output; synchronous.  Workspace as laue_sinkhorn. */
typedef struct laue_objective {
    double mass, cost_inlier, cost_total, entropy, sem_objective;
} laue_objective;

int laue_objectives(const laue_geometry *geom, const laue_obs_spots *obs,
                    const laue_model_spots *model, const laue_ot_params *par,
                    const laue_potentials *pot, double sigma_mm, laue_objective *out,
                    void *ws, size_t ws_bytes, void *stream);

/* Dense plan block b: Q[i][j] = exp((f_i + g_j - c_ij)/eps) for the
 * detected x model spots of block b, row-major FP32 [I_b][J_b] (device).
 * For tests and small problems. */
int laue_plan_block(const laue_geometry *geom, const laue_obs_spots *obs,
                    const laue_model_spots *model, const laue_ot_params *par,
                    const laue_potentials *pot, int32_t block, float *Q, void *stream);

/* Dense cost block b: C[i][j] = c_ij = D^2 ||rhat_ij - r_j||^2 (mm^2,
 * Sec. 4, the likelihood L_ij up to a constant and the factor -1/(2 sigma^2))
 * for the detected x model spots of block b, row-major FP32 [I_b][J_b]
 * (device), computed exactly as the streamed passes compute it.  For tests
 * and small problems. */
int laue_cost_block(const laue_geometry *geom, const laue_obs_spots *obs,
                    const laue_model_spots *model, double distance, int32_t block, float *C,
                    void *stream);

/* ---- M-step: per-grain weighted Gauss-Newton ----------------------------- */

typedef struct laue_gn_params {
    int32_t k_gn;               /* Gauss-Newton steps (method 0) or coordinate-descent
                                 * sweeps (method 1) with the plan held fixed */
    double mu_rel;              /* Levenberg term mu = mu_rel * tr(H) / 6 (method 0) */
    /* 0: joint Gauss-Newton on (R, x); 1: the paper's coordinate descent
     * (App. B, Alg. LaueOT's M-step): per sweep, LauePosNewton on x with R
     * fixed (Eqs. xgrad, xhess; x <- x - H^-1 g, at most k_newton steps,
     * a grain stops after the step with |dx| < tol_x mm), then LaueRotMM on R
     * at the new x (Eqs. M0, Mm, majmin_step: M0 summed per plane, shifted by
     * |smallest eigenvalue| when negative, R <- Wahba(M_m R w_m, w_m, 1) until
     * ||R' - R||_F < tol_r or k_mm steps).  Wahba's problem is solved by
     * Davenport's q-method (the same minimiser as the SVD of Alg. Wahba). */
    int32_t method;
    int32_t k_newton;           /* method 1: Newton steps per sweep (>= 1) */
    int32_t k_mm;               /* method 1: MM steps per sweep (>= 1) */
    double tol_x;               /* method 1: Newton stop, mm (>= 0) */
    double tol_r;               /* method 1: MM stop, Frobenius norm (>= 0) */
} laue_gn_params;

/* M-step (Eq. mstep_obj): the plan Q is given by (pot, par->eps) and the
 * model spots' current geometry (the E-step state).  Method 0: each of k_gn
 * steps re-evaluates the model spots at the current grains, forms per grain
 * the FP64 normal equations H = sum Q J^T J + mu I, g = sum Q J^T rho with
 * rho = D (rhat - r), and applies R <- exp([omega]_x) R, x <- x + dx with
 * (omega, dx) = -H^-1 g.  Method 1: k_gn sweeps of LauePosNewton then
 * LaueRotMM (see laue_gn_params); a Newton step whose 3x3 Hessian is
 * singular is skipped.  Grains without weight stay unchanged.  step_norm:
 * optional device FP64 [n_grains], |(omega, dx)| of the last step (method
 * 0) or |dx| of the last Newton step (method 1).  Method 1 needs
 * planes->n <= 1024. */
int laue_mstep(const laue_geometry *geom, const laue_planes *planes,
               const laue_obs_spots *obs, laue_model_spots *model,
               const laue_ot_params *par, const laue_potentials *pot,
               const laue_gn_params *gn, laue_grains *grains, double *step_norm,
               void *ws, size_t ws_bytes, void *stream);

/* ---- EM driver (Alg. LaueOT) ---------------------------------------------- */

typedef struct laue_em_params {
    laue_ot_params ot;          /* eps is ignored: schedule below */
    laue_gn_params gn;
    double eps_start, eps_end;  /* geometric schedule over n_stages stages */
    int32_t n_stages;
    int32_t iters_per_stage;
    /* how the Sinkhorn passes are issued between host polls: 1 direct kernel
     * launches, 2 replay of a captured hipGraph of one polling chunk, 0 tune:
     * time both on chunks in which every pass does work and keep the faster;
     * with ot.chunk == 0 the chunk of each temperature stage is sized from the
     * iterations that stage needed in the previous EM iteration */
    int32_t launch;
    /* tile shape of the Sinkhorn passes: 1 one detected (model) spot per lane,
     * 2 two per lane sharing each streamed load, 0 tune per temperature stage
     * (in the first Sinkhorn of a stage, row pass 2 is timed in shape 1 and
     * row pass 3 in shape 2, and the faster kept; shape 1 when a sample
     * converges within those iterations); every shape gives the same result */
    int32_t tile;
    /* annealing (Sec. 5.1, Alg. LaueOT).  eps_cool = 0: the stage schedule
     * above.  0 < eps_cool < 1: the paper's cooling: the first EM iteration
     * runs at eps_start and the temperature is multiplied by eps_cool after
     * every iteration while it is above eps_end, i.e. the temperatures
     * eps_start eps_cool^k, k = 0 .. K, K the first k with eps_start
     * eps_cool^k <= eps_end (products taken in that order in FP64; n_stages and
     * iters_per_stage are not read); then at most final_iters more EM
     * iterations at the last temperature, stopping after the first iteration
     * (from iteration K on) whose plan differs from the previous iteration's by
     * zeta = ||Q^{k+1} - Q^k||_F <= zeta_tol over the detected x model entries
     * and the bins (zeta_tol <= 0: every final iteration runs).  zeta is
     * evaluated in FP32 per entry (a floor near 1e-7 sqrt(entries with
     * Q > 0)).  With the sparse assignment (ot.rho > 0) the plans are 0 off
     * each detected spot's rho neighbours, which each E-step chooses anew:
     * zeta runs over the union of the two E-steps' neighbour sets.  The
     * plan-change test runs in laue_em and laue_index (one sample). */
    double eps_cool;
    int32_t final_iters;
    double zeta_tol;
    /* > 0: laue_em_stats.objective receives the FP64 summaries of the last
     * E-step's plan (laue_objectives) with the paper-unit objective at this
     * spot noise (mm); 0: not computed */
    double sigma_mm;
} laue_em_params;

typedef struct laue_em_stats {
    int32_t n_em_iter;
    int64_t sinkhorn_iters;     /* total over the run */
    int64_t cost_entries;       /* same-block (i,j) pairs streamed, all passes */
    int32_t not_converged;      /* EM iterations whose Sinkhorn hit the cap */
    double last_err;
    /* GPU time measured with HIP events on the call's stream (ms) and the
     * work it covers: Sinkhorn row/column passes, M-step passes. */
    double sinkhorn_ms;
    int64_t sinkhorn_passes;
    int64_t sinkhorn_entries;
    double mstep_ms;
    int64_t mstep_entries;
    int32_t launch_used;        /* 1 direct launches, 2 graph replay */
    int32_t polls;              /* host polls of the Sinkhorn control blocks */
    int32_t tile2_solves;       /* Sinkhorn solves run in the two-per-lane shape */
    /* the likelihood out (Eqs. elbo, estep_obj): FP64 summaries of the last
     * E-step's plan (laue_objectives of its potentials and geometry) when
     * laue_em_params.sigma_mm > 0, else NaN */
    laue_objective objective;
    double zeta;                /* cooling mode, dense: ||Q^{k+1} - Q^k||_F of the last
                                 * EM iteration (NaN when not evaluated) */
    int32_t final_iters_run;    /* cooling mode: EM iterations after the cooling */
} laue_em_stats;

/* Hard assignments of the EM's last E-step plan (Alg. LaueOT's output Q:
 * its potentials and the model-spot geometry of that E-step, i.e. before the
 * last M-step moves the grains).  Per detected spot (device [n_obs], the four
 * arrays all given or all NULL): j_star = argmax over its block's model spots
 * and the outlier column of Q (lowest index on ties; -1 for the outlier
 * column), its grain (-1 for outlier), q_star = Q_ij*, q_out = Q_i0.  Under
 * unbalanced or partial OT (no outlier column) q_out is the mass the plan
 * leaves untransported, max(0, 1 - sum_j Q_ij), and takes the outlier
 * column's place in the comparison.  Per model spot (device [n_model], may be
 * NULL): q_unm = Q_0j, its entry in the unmatched row (Eq. update_L; the
 * weight behind the unmatched-spot rule of Sec. 6.2); 0 under unbalanced or
 * partial OT. */
typedef struct laue_assignments {
    int32_t *j_star;
    int32_t *grain;
    float *q_star;
    float *q_out;
    float *q_unm;
} laue_assignments;

/* Full EM: for each stage s and iteration: forward eval -> Sinkhorn (warm
 * started) -> M-step.  The model-spot list is frozen.  pot: in = warm start
 * (zeros for Alg. BalancedOT's x = y = 1), out = final.  Synchronous. */
int laue_em(const laue_geometry *geom, const laue_planes *planes,
            const laue_obs_spots *obs, laue_model_spots *model,
            const laue_em_params *par, laue_grains *grains, laue_potentials *pot,
            laue_assignments *assign, laue_em_stats *stats,
            void *ws, size_t ws_bytes, void *stream);

/* The neighbour sets of the sparse assignment (Sec. 5.2), as the sparse
 * Sinkhorn builds them: for every detected spot the par->rho nearest model
 * spots of its block by the chord cost, ordered by (cost, index), ties to the
 * lower index.  nbr [n_obs x rho] (device int32, model-spot index or -1 when
 * the block has fewer model spots), cost [n_obs x rho] (device FP32, c_ij in
 * mm^2; +inf past the last neighbour), n_pairs (host, may be NULL) the kept
 * pairs.  Only par->distance and par->rho are read.  Workspace:
 * laue_sparse_workspace_size with n = 1. */
int laue_sparse_neighbors(const laue_geometry *geom, const laue_obs_spots *obs, const laue_model_spots *model,
                          const laue_ot_params *par, int32_t *nbr, float *cost, int64_t *n_pairs, void *ws,
                          size_t ws_bytes, void *stream);

/* The first temperature of the sparse assignment (Sec. 7: chosen so that the
 * farthest of the rho neighbours keeps a non-negligible probability at the
 * start): the median over detected spots of the chord cost to their farthest
 * kept neighbour (laue_sparse_neighbors; spots of blocks without model spots
 * left out; the mean of the two middle values for an even count), divided by
 * ln 100, i.e. that neighbour's Gibbs weight relative to a zero-cost match is
 * 1/100 for the median spot.  *eps_init (HOST) in mm^2; 1.0 when no detected
 * spot has a neighbour.  Only par->distance and par->rho (8, 16 or 32) are
 * read.  Workspace: laue_sparse_workspace_size with n = 1.  Synchronous. */
int laue_eps_init(const laue_geometry *geom, const laue_obs_spots *obs, const laue_model_spots *model,
                  const laue_ot_params *par, double *eps_init, void *ws, size_t ws_bytes, void *stream);

/* Workspace of laue_sinkhorn, laue_mstep and laue_em (n = 1) or
 * laue_em_batched (n samples) when ot.rho > 0: the dense workspace plus the
 * neighbour sets (rho int + float per detected spot), the filter's candidate
 * lists (8 rho per detected spot) and the column lists.  0 on bad input. */
size_t laue_sparse_workspace_size(int32_t n, const laue_geometry *geoms, const int64_t *n_obs,
                                  const int64_t *n_model, const int32_t *n_grains, int32_t rho);

/* Batched EM of n independent samples (arrays of n structs, one per sample;
 * each sample's device arrays are its own).  Every pass of the E- and M-steps
 * is one launch over the work of all samples; each sample keeps its own bins,
 * temperature schedule, convergence and statistics, and gets the result that
 * laue_em would give it alone.  Samples share n_stages, iters_per_stage and
 * gn.k_gn, launch and ot.chunk.  assigns may
 * be NULL or hold NULL arrays for some samples.  The millisecond fields of
 * every stats entry are the batch's totals.  Synchronous; LAUE_ENOCONV when
 * some Sinkhorn of some sample stopped at its cap. */
size_t laue_em_batched_workspace_size(int32_t n, const laue_geometry *geoms, const int64_t *n_obs,
                                      const int64_t *n_model, const int32_t *n_grains);
int laue_em_batched(int32_t n, const laue_geometry *geoms, const laue_planes *planes,
                    const laue_obs_spots *obs, laue_model_spots *models, const laue_em_params *pars,
                    laue_grains *grains, laue_potentials *pots, laue_assignments *assigns,
                    laue_em_stats *stats, void *ws, size_t ws_bytes, void *stream);

/* ---- prototype scoring (Sec. 6, App. D-E) -------------------------------- */

/* Spot-pair candidate orientations.  Each detected spot of a pair is read as
 * a reflection of a grain at the sample centre: its ray rhat = p/|p| gives the
 * lab normal u = (e - rhat)/|e - rhat| and sin(theta) = u.e (Eqs. ray_r, bragg),
 * the sample-frame normal n = Gamma_t^T u.  Pair k is drawn with Philox4x32-10
 * (counter (k, 0, 0, 5), key = seed): word 0 mod n_rot picks the rotation,
 * words 1 and 2 mod (spots of that rotation) the two spots (a == b: none).
 * Hypotheses: plane m_a among one representative per orbit of the 24 proper
 * cubic rotations (the first plane of each orbit in list order) and any
 * non-parallel plane m_b, both with
 * 2 d sin(theta) in band, the angle between their normals within delta of the
 * angle between n_a and n_b; the orientation solves Wahba's problem (App. A)
 * for (n_a, w_a), (n_b, w_b), (n_a x n_b, w_a x w_b) (Davenport's q-method,
 * FP64).  Position hypothesis x = 0.  Ordered by (pair, m_a, m_b). */
typedef struct laue_cand_params {
    int64_t n_pairs;
    uint64_t seed;
    double delta_deg;
    /* optional explicit pairs (device [n_pairs] detected-spot indices, both
     * NULL for the random draw); a pair whose spots are out of range or not of
     * one rotation yields no hypothesis */
    const int32_t *pair_a, *pair_b;
} laue_cand_params;

/* Candidate outputs (device; capacity n on entry, count written on return;
 * every array except q may be NULL).  feat: [n][16] FP32 features
 * (0 cos(n_a,n_b), 1 cos(w_a,w_b), 2 |angle difference|/delta, 3-4 sin theta,
 * 5-6 wavelength within the band, 7-8 N/N_max, 9 |p_a - p_b|/(2 l),
 * 10-11 |(p1,p2)|/l, 12-13 detector ids, 14-15 cheap support, see
 * laue_candidate_support). */
typedef struct laue_candidates {
    int64_t n;
    double *q;
    int32_t *pair, *ma, *mb, *spot_a, *spot_b;
    float *feat;
} laue_candidates;

size_t laue_candidates_workspace_size(const laue_geometry *geom, int32_t n_planes, int64_t n_pairs);

/* Generates the hypotheses of pairs 0 .. n_pairs-1.  *n_found (HOST) is the
 * total; out->n becomes min(total, capacity) and the first ones are written.
 * Synchronous. */
int laue_candidates_generate(const laue_geometry *geom, const laue_planes *planes,
                             const laue_obs_spots *obs, const laue_cand_params *par,
                             laue_candidates *out, int64_t *n_found, void *ws, size_t ws_bytes,
                             void *stream);

/* Single-grain refinement and scoring of candidate grains (App. D-E).
 * Refinement: k_refine iterations on the temperature schedule eps_start ->
 * eps_end (geometric), each a row-softmax E-step over the candidate's frozen
 * model spots plus the outlier column (Eq. elbo_single), then k_gn
 * Gauss-Newton steps with Q fixed.  Scoring at the refined grain: a model
 * spot is unmatched when no detected spot of its block is within c_out; a
 * candidate is kept when unmatched < f_out * model spots; kept candidates
 * get SPOT entries Lbar_in = ln sum_j exp(-c_ij / (2 sigma^2)) for every
 * detected spot i of a block where the sum exceeds exp(-c_out / (2 sigma^2))
 * (the outlier floor).  Candidates run in batches of `chunk`; a batch holds
 * at most chunk * max_spots_per_cand model spots. */
typedef struct laue_score_params {
    double sigma_mm, distance, c_out, f_out;
    double eps_start, eps_end;
    int32_t k_refine, k_gn;
    double mu_rel;
    int32_t chunk, max_spots_per_cand;
    /* 0: the geometric schedule eps_start -> eps_end above; in (0, 1]:
     * Alg. SingleLaueOT's cooling, iteration k at eps_start eps_cool^k
     * (k = 0 .. k_refine - 1, FP64 products in order; eps_end not read) */
    double eps_cool;
    /* refinement passes: 0 skips only the pairs whose plan term is 0 in FP32
     * (the result is that of evaluating every pair); d > 0 also skips pairs
     * whose term exp(-c / eps) is below 2^-d times the outlier bin's
     * exp(-c_out / eps), i.e. below 2^-d of the row's softmax normaliser
     * (which starts at the bin term and only grows): each such row weight is
     * < 2^-d, and for d >= 26 the term is below a quarter of the normaliser's
     * FP32 ulp, so the normalisers are those of evaluating every pair (the
     * binding's default: d = 26) */
    double drop_log2;
} laue_score_params;

/* Scoring outputs (device).  n_model, n_unmatched, keep: [n_cand] (may be
 * NULL).  SPOT matrix as CSR by candidate: lbar_off [n_cand + 1], lbar_row,
 * lbar_val [lbar_cap]; lbar_n (out) entries.  Within a candidate the entries
 * are grouped by block; within a block their order is the scoring pass's
 * (deterministic, not by row).  The scoring passes (unmatched filter, SPOT
 * entries, Sec. 6.2 and App. E) read the detected spots through the cell
 * index below: per model spot, the detected spots within a radius beyond
 * which its cost exceeds c_out and its term of a row's sum is below half the
 * floor over the block's model spots of the candidate: skipping the others
 * changes neither the entries nor the unmatched counts. */
typedef struct laue_score_out {
    int32_t *n_model;
    int32_t *n_unmatched;
    uint8_t *keep;
    int64_t *lbar_off;
    int32_t *lbar_row;
    float *lbar_val;
    int64_t lbar_cap;
    int64_t lbar_n;
    int64_t pairs_streamed;   /* (out) same-block (detected, model) pairs of all
                               * passes: the work the method defines */
    int64_t pairs_evaluated;  /* (out) of those, the pairs the passes evaluate:
                               * the refinement passes' (see below) and the
                               * scoring passes' (the detected spots within
                               * each model spot's scoring radius, times the
                               * slot's model spots) */
    int64_t pairs_refine;     /* (out) the refinement passes' share of pairs_streamed */
} laue_score_out;

/* The refinement passes read each block's detected spots through a cell
 * index (a 32 x 32 grid over the block's bounding box, spots sorted stably by
 * cell): a (block, candidate) pass evaluates only the spots of the cells
 * within R_j of one of the candidate's model spots s_j, where R_j is the
 * detector distance beyond which the plan term exp(-c / eps) of model spot j
 * is 0 in FP32 (from c' >= t^2 v_n^2 / (2 |v|^2), t = |delta| / (|v| + |delta|),
 * a bound that holds for every detected spot delta away in the detector
 * plane).  The skipped pairs add exactly 0 to every sum.  n_obs (the
 * detected spots of the calls) sizes the index; n_obs < 2^31. */
size_t laue_score_workspace_size(const laue_geometry *geom, int64_t n_obs, const laue_score_params *par);

/* Refines the candidates in place (q, x) and scores them.  Returns
 * LAUE_ECAPACITY if a batch or the SPOT output overflows.  Synchronous. */
int laue_score_candidates(const laue_geometry *geom, const laue_planes *planes,
                          const laue_obs_spots *obs, laue_grains *cand,
                          const laue_score_params *par, laue_score_out *out, void *ws,
                          size_t ws_bytes, void *stream);

size_t laue_spot_greedy_workspace_size(int32_t n_cand, int64_t n_rows);

/* Greedy SPOT prototype selection (Alg. LaueSpotGreedy) on a sparse Lbar with
 * floor phi: f(S) = sum_i max(phi, max_{n in S} Lbar_in) - |I| phi; each step
 * adds the candidate of largest increment (lowest index on ties) until k_max
 * or no increment is left.  picks [k_max], gains [k_max] (device, FP64
 * increments Delta_k); *n_picked (HOST).  Synchronous.
 * Increments computed at an earlier step bound the current ones from above
 * (covers only rise): each step recomputes, grid-wide, only the candidates
 * whose bound reaches the best exact increment, so the picks and increments
 * are those of recomputing every increment at every step.
 * laue_spot_greedy_workspace_size is the minimum; with 8 bytes per SPOT entry
 * beyond it (and lbar_off[0] = 0) the entries are copied there and each
 * recomputation drops the entries that can no longer add to an increment
 * (the picks and increments do not change, bit for bit). */
int laue_spot_greedy(const int64_t *lbar_off, const int32_t *lbar_row, const float *lbar_val,
                     int32_t n_cand, int64_t n_rows, double phi, int32_t k_max, int32_t *picks,
                     double *gains, int32_t *n_picked, void *ws, size_t ws_bytes, void *stream);

/* ---- learned proposal: a small network that ranks candidates ------------ */

/* Cheap support of candidates (features 14 and 15).  The candidate grain,
 * placed at the sample centre (the position hypothesis of the spot-pair
 * candidates), predicts the reflections of the first n_support_planes planes
 * of the list that have no lower-order parallel plane (forward model of
 * Sec. 3.3: wavelength in band, tau > 0, strictly inside the detector) at the
 * probe rotations t_k = (t + floor(k T / 3)) mod T, k = 1, 2, where t is the
 * rotation of the candidate's spot_a.  A prediction is hit when a detected
 * spot of the same (rotation, detector) block lies within radius_mm (<=).
 * feat[16 c + 13 + k] = hits / max(predictions, 1).  FP64 geometry. */
typedef struct laue_support_params {
    double radius_mm;
    int32_t n_support_planes;
} laue_support_params;

size_t laue_candidate_support_workspace_size(const laue_geometry *geom, int32_t n_planes,
                                             int64_t n_obs, const laue_support_params *par);
/* cand: q, spot_a and feat are read / written (device); asynchronous. */
int laue_candidate_support(const laue_geometry *geom, const laue_planes *planes,
                           const laue_obs_spots *obs, const laue_candidates *cand,
                           const laue_support_params *par, void *ws, size_t ws_bytes,
                           void *stream);

/* Training labels of candidates drawn on simulated spots: label[c] = 1 when
 * both spots of the pair come from one true grain g (spot_grain [n_obs],
 * -1 for outliers, device) and the candidate orientation is within max_deg
 * of truth->q[g] up to the 24 proper cubic rotations; else 0.  mis_deg
 * (may be NULL) receives that misorientation (degrees; +inf when the spots
 * are not from one grain).  Device outputs [cand->n]; asynchronous. */
int laue_candidate_labels(const laue_candidates *cand, const int32_t *spot_grain, int64_t n_obs,
                          const laue_grains *truth, double max_deg, float *label, float *mis_deg,
                          void *stream);

/* Training labels by the nearest true grain: label[c] = 1 when the candidate
 * orientation is within max_deg of some truth->q[g] up to the 24 proper cubic
 * rotations, whichever spots its pair came from (single-grain refinement from
 * such a start reaches the grain; farther starts seldom do).  mis_deg and
 * nearest (may be NULL) receive the smallest misorientation (degrees) and its
 * grain (lowest index on ties; -1 without true grains).  FP64.  Device
 * outputs [cand->n]; only cand->q is read; asynchronous. */
int laue_candidate_labels_nearest(const laue_candidates *cand, const laue_grains *truth, double max_deg,
                                  float *label, float *mis_deg, int32_t *nearest, void *stream);

/* Same-grain spot pairs for training the proposal on simulated spots.  Pair k
 * draws Philox4x32-10 counter (k, 0, 0, 7) under the key (seed low, seed
 * high): a = x0 mod n_obs; if spot a is an outlier (spot_grain -1) or no
 * other spot of its grain lies in its rotation (either detector), the pair is
 * (-1, -1); else b is the (x1 mod count)-th of those spots in index order.
 * out_a, out_b [n_pairs] (device).  Asynchronous. */
int laue_pairs_same_grain(const laue_geometry *geom, const laue_obs_spots *obs,
                          const int32_t *spot_grain, int64_t n_pairs, uint64_t seed,
                          int32_t *out_a, int32_t *out_b, void *ws, size_t ws_bytes, void *stream);
size_t laue_pairs_same_grain_workspace_size(const laue_geometry *geom);

size_t laue_select_top_workspace_size(int64_t n);
/* Indices of the k largest of score [n] (device, n < 2^31), equal scores in
 * increasing index order (-0 equals +0), NaN below everything; written ascending to
 * out [k] (device).  Asynchronous. */
int laue_select_top(const float *score, int64_t n, int64_t k, int32_t *out, void *ws,
                    size_t ws_bytes, void *stream);

/* 16-256-256-1 perceptron (ReLU, sigmoid output) on the 16 candidate
 * features.  params: FP32 masters, layout W1 [256][16], b1 [256],
 * W2 [256][256], b2 [256], w3 [256], b3 [1] (laue_mlp_n_params entries);
 * wbf16: bfloat16 copies of W1, W2, W2^T and w3 (laue_mlp_n_bf16 entries),
 * refreshed by laue_mlp_init / laue_mlp_adam / laue_mlp_sync_bf16.  Weights and
 * the activations entering each product are rounded to bfloat16 (nearest
 * even); products run on the matrix cores with FP32 accumulation.  adam_m,
 * adam_v: FP32 moments (training only); step: Adam step count.  All device. */
typedef struct laue_mlp {
    int32_t n_in;
    int32_t n_hidden;
    float *params;
    uint16_t *wbf16;
    float *adam_m, *adam_v;
    int32_t step;
} laue_mlp;

typedef struct laue_adam_params {
    double lr, beta1, beta2, eps;
} laue_adam_params;

int64_t laue_mlp_n_params(int32_t n_in, int32_t n_hidden);
int64_t laue_mlp_n_bf16(int32_t n_in, int32_t n_hidden);

/* He-uniform weights from Philox4x32-10 (counter (i, 0, 0, 6)), zero biases,
 * output layer scaled by 0.1; step = 0.  Adam moments are not touched. */
int laue_mlp_init(laue_mlp *m, uint64_t seed, void *stream);
int laue_mlp_sync_bf16(laue_mlp *m, void *stream);

size_t laue_mlp_forward_workspace_size(int64_t n);
/* prob[i] = sigmoid(network(feat[i])) for feat [n][16] FP32 (device). */
int laue_mlp_forward(const laue_mlp *m, const float *feat, int64_t n, float *prob, void *ws,
                     size_t ws_bytes, void *stream);

size_t laue_mlp_train_workspace_size(int64_t batch);
/* Gradient of the mean binary cross-entropy over a batch (batch % 16 == 0)
 * into grad [n_params] (device, may be NULL) and the loss (HOST).  Synchronous. */
int laue_mlp_backward(const laue_mlp *m, const float *feat, const float *label, int64_t batch,
                      float *grad, double *loss, void *ws, size_t ws_bytes, void *stream);
/* One Adam step (bias-corrected) on the masters, then the bf16 copies. */
int laue_mlp_adam(laue_mlp *m, const float *grad, const laue_adam_params *ap, void *stream);
/* backward + Adam. */
int laue_mlp_train_step(laue_mlp *m, const float *feat, const float *label, int64_t batch,
                        const laue_adam_params *ap, double *loss, void *ws, size_t ws_bytes,
                        void *stream);

/* One training epoch over examples feat [n][16], label [n] (device): the
 * floor(n / batch) batches of a seeded permutation, each gathered by the
 * library and taken through laue_mlp_train_step's kernels (backward, Adam).
 * The order: example i gets the 64-bit key (x0 << 32) | x1 of Philox4x32-10
 * counter (i, epoch, 0, 8) under the key (seed low, seed high), and the
 * examples are visited by increasing key (a stable radix sort: equal keys by
 * index); the last n mod batch of that order are left out.  *loss_mean (HOST)
 * is the mean binary cross-entropy over the visited examples (each batch's
 * before its Adam step).  batch % 16 == 0, batch <= n < 2^31.
 * Synchronous. */
size_t laue_mlp_epoch_workspace_size(int64_t n, int64_t batch);
int laue_mlp_train_epoch(laue_mlp *m, const float *feat, const float *label, int64_t n, int64_t batch,
                         uint64_t seed, int32_t epoch, const laue_adam_params *ap, double *loss_mean,
                         void *ws, size_t ws_bytes, void *stream);

/* ---- Sobol-grid starts (Sec. 6.1) ------------------------------------------ */

/* Starts of single-grain fitting from a Sobol sequence over the six
 * dimensions (R, x) (Sec. 6.1): point n (Antonov-Saleev order: XOR of the
 * direction numbers over the bits of the Gray code of n; Joe and Kuo's
 * direction numbers for dimensions 2..6), u in [0, 1)^6; orientation from the
 * modified Rodrigues parameters p = (2 u_1..3 - 1) mrp_half, q = ((1 - |p|^2),
 * 2 p) / (1 + |p|^2); position x = (2 u_4..6 - 1) x_half.  With restrict_fz
 * only orientations in the cubic (432) fundamental zone are kept: Rodrigues
 * vector r = q_1..3 / q_0 with |r_i| <= tan(pi/8) and |r_1|+|r_2|+|r_3| <= 1
 * (the crystal symmetry restriction of Sec. 6.1). */
typedef struct laue_sobol_params {
    int64_t first;              /* index of the first point (0 is the origin) */
    double mrp_half;            /* half side of the MRP cube; 0: tan(pi/16), the
                                 * largest MRP component in the cubic zone */
    double x_half[3];           /* half extents of the position box (mm) */
    int32_t restrict_fz;        /* 1: keep orientations in the cubic zone only */
} laue_sobol_params;

size_t laue_sobol_workspace_size(int64_t n_points);

/* Points first .. first + n_points - 1 (n_points < 2^31, indices < 2^32): the
 * kept ones, in index order, to q [n_kept][4] (q_0 > 0) and x [n_kept][3]
 * (device FP64, capacity n_points); *n_kept (HOST).  Synchronous. */
int laue_sobol_starts(const laue_sobol_params *par, int64_t n_points, double *q, double *x,
                      int64_t *n_kept, void *ws, size_t ws_bytes, void *stream);

/* ---- end-to-end indexing ------------------------------------------------- */

#define LAUE_INDEX_PLAIN 0      /* every candidate is refined and scored */
#define LAUE_INDEX_LEARNED 1    /* the network keeps the best-scored fraction */
#define LAUE_INDEX_SOBOL 2      /* Sobol-grid starts (Sec. 6.1) in place of spot pairs:
                                 * max_candidates points from sobol, the kept ones
                                 * refined from their own (q, x) and scored */

/* The multigrain solve (Sec. 6, Alg. MultiGrainLaueOT) from detected spots:
 *   1. spot-pair candidates (laue_candidates_generate; at most max_candidates
 *      of them, the first ones, are kept);
 *   2. learned mode: support features (laue_candidate_support), the network
 *      (laue_mlp_forward), the ceil(top_frac * n) best (laue_select_top);
 *   3. single-grain refinement and scoring (laue_score_candidates, x = 0 start);
 *   4. greedy SPOT (laue_spot_greedy, floor -c_out / (2 sigma^2), at most k_max
 *      picks) and k* where f, the running sum of the increments Delta, bends
 *      most (Eq. spot_ngrains' second difference over h = 8 picks): the
 *      argmax over k >= 1 of the mean Delta of the m = min(k, 8) picks up to k
 *      minus the mean of the 8 picks after k (Delta beyond the picks is 0);
 *      the first k* picks are the prototypes;
 *   5. the harmonic-merged model spots of the prototypes, frozen (Sec. 4.2),
 *      and the EM of laue_em from zero potentials with
 *      T_b = max(ceil(t_b_frac |J|), |J| - |I|).
 * Capacities bound the workspace: max_candidates, lbar_cap SPOT entries,
 * k_max prototypes, max_model_spots; an overflow returns LAUE_ECAPACITY. */
typedef struct laue_index_params {
    int32_t mode;
    laue_cand_params cand;          /* pair_a / pair_b must be NULL */
    int64_t max_candidates;
    const laue_mlp *mlp;            /* learned mode */
    laue_support_params support;    /* learned mode */
    double top_frac;                /* learned mode */
    laue_score_params score;
    int64_t lbar_cap;
    int32_t k_max;
    int64_t max_model_spots;
    double t_b_frac;
    laue_em_params em;              /* em.ot.t_b is set from t_b_frac; with em.eps_cool > 0 and
                                     * em.eps_start <= 0 the first temperature is laue_eps_init
                                     * of the prototypes' model spots (rho = em.ot.rho, or 32) */
    laue_sobol_params sobol;        /* Sobol mode */
} laue_index_params;

/* Per-stage wall-clock times (ms, host clock around each synchronous stage)
 * and sizes. */
typedef struct laue_index_stats {
    int64_t n_candidates_found, n_candidates, n_scored, lbar_entries;
    int32_t n_picked, n_prototypes;
    int64_t n_model_spots;
    double ms_candidates, ms_proposal, ms_score, ms_greedy, ms_em, ms_total;
    laue_em_stats em;
    int64_t score_pairs;            /* same-block pairs of the scoring stage (laue_score_out.pairs_streamed) */
    int64_t score_pairs_evaluated;  /* of those, the pairs evaluated (laue_score_out.pairs_evaluated) */
    int64_t score_pairs_refine;     /* the refinement passes' share (laue_score_out.pairs_refine) */
} laue_index_stats;

/* Output grains (device, capacity >= k_max; n_grains = k* on return) and the
 * per-detected-spot assignments of the final EM's last E-step (j_star, grain,
 * q_star, q_out: all four arrays or none; q_unm is not written, the model
 * spots of the EM living in the workspace).  The likelihood of that plan
 * (Eqs. elbo, estep_obj) is stats->em.objective, at em.sigma_mm or, when that
 * is 0, at score.sigma_mm. */
typedef struct laue_index_out {
    int32_t capacity;
    int32_t n_grains;
    double *q, *x;
    laue_assignments assign;
} laue_index_out;

size_t laue_index_workspace_size(const laue_geometry *geom, int32_t n_planes, int64_t n_obs,
                                 const laue_index_params *par);
/* Synchronous.  Returns LAUE_ENOCONV (a warning) when an EM Sinkhorn stopped
 * at its cap. */
int laue_index(const laue_geometry *geom, const laue_planes *planes, const laue_obs_spots *obs,
               const laue_index_params *par, laue_index_out *out, laue_index_stats *stats,
               void *ws, size_t ws_bytes, void *stream);

/* laue_index of n independent samples in one call (arrays of n, one entry per
 * sample; each sample's device arrays, outputs and parameters are its own;
 * the samples share em.ot.rho).  Stages 1-4 and the prototypes' model spots
 * run sample by sample (each of those stages fills the GPU on its own); the
 * final EM of every sample with prototypes then runs as one batch
 * (laue_em_batched: one launch per pass over all samples) when the samples'
 * EM parameters allow it (same n_stages, iters_per_stage, gn.k_gn, launch,
 * tile, ot.chunk, eps_cool, final_iters and number of temperatures, and no
 * plan-change stop), else sample after sample.  Every sample gets the grains,
 * assignments and statistics that laue_index gives it alone; the EM and
 * total milliseconds are the batch's.  Workspace: one region the size of the
 * largest laue_index workspace or of the batched EM's at the capacities
 * (max_model_spots, k_max), whichever is larger, plus each sample's model
 * spots and potentials.  Synchronous; LAUE_ENOCONV when an EM Sinkhorn of
 * some sample stopped at its cap. */
size_t laue_index_batched_workspace_size(int32_t n, const laue_geometry *geoms, const int32_t *n_planes,
                                         const int64_t *n_obs, const laue_index_params *pars);
int laue_index_batched(int32_t n, const laue_geometry *geoms, const laue_planes *planes,
                       const laue_obs_spots *obs, const laue_index_params *pars, laue_index_out *outs,
                       laue_index_stats *stats, void *ws, size_t ws_bytes, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* LAUEOT_H */
