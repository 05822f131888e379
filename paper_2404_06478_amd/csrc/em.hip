// E-step (streamed log-domain Sinkhorn with outlier row/column), M-step
// (per-grain weighted Gauss-Newton) and the EM driver.
//
// Paper: Sec. 4.2-4.4 (Eqs. update_L, elbo, estep_obj, mstep_obj),
// Alg. BalancedOT and Alg. LaueOT.
//
// Data layout (all device, caller memory unless "ws"):
//   detected spots  P1, P2           block-sorted FP32 SoA
//   model spots     Col8 cols (ws)   32-byte packed columns, block-sorted
//   potentials      F (2 buffers: caller's f and one in ws), G in place
//   control         SinkCtl (ws)     bin potentials, iteration, flags
// A pass is a grid of one-wave workgroups; each owns 64 rows (row pass) or
// 64 columns (column pass) of one (rotation, detector) block and streams the
// other side of that block through scalar loads, so the |I_b| x |J_b| cost
// block is recomputed on the fly and never stored.
#include <algorithm>
#include <cmath>
#include <numeric>

#include "common.h"

namespace laue {

int launch_pack(const laue_model_spots *m, Col8 *cols, hipStream_t s);


struct Item {
    int r0, r1, c0, c1;
};

struct SinkCtl {
    double f0[2], g0[2];   // bin potentials of states with even / odd index
    double cs_sum;         // sum_j exp((f0 + g_j - c_unm)/eps) of the latest g
    double err;
    double eps, kexp;      // eps and log2(e)/eps
    int iter;              // completed row passes
    int done;
    int final_state;
    int converged;
    unsigned ticket;
    int best_iter;         // iteration of the last 1% improvement of the error
    int pad[2];
    double best_err;
};

struct SinkParams {
    double c_out, c_unm, c_sink, t_a, t_b, tol;
    float twoD2;
    int n_max;
};

// ---------------------------------------------------------------- helpers

__device__ __forceinline__ bool last_block(SinkCtl *ctl) {
    __shared__ int is_last;
    __threadfence();
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned t = atomicAdd(&ctl->ticket, 1u);
        is_last = (t == gridDim.x - 1) ? 1 : 0;
    }
    __syncthreads();
    if (is_last) __threadfence();
    return is_last != 0;
}

__global__ void k_ctl_init(SinkCtl *ctl, double f0, double g0, double eps) {
    ctl->f0[0] = f0;
    ctl->g0[0] = g0;
    ctl->f0[1] = f0;
    ctl->g0[1] = g0;
    ctl->cs_sum = 0.0;
    ctl->err = INFINITY;
    ctl->eps = eps;
    ctl->kexp = 1.4426950408889634 / eps;
    ctl->iter = 0;
    ctl->done = 0;
    ctl->best_iter = 0;
    ctl->best_err = INFINITY;
    ctl->final_state = 0;
    ctl->converged = 0;
    ctl->ticket = 0u;
}

// cs_sum of the initial state: sum_j exp((f0 + g_j - c_unm)/eps).
__global__ __launch_bounds__(64) void k_cs_init(const float *__restrict__ G, int64_t nJ,
                                                SinkCtl *ctl, double *__restrict__ part,
                                                SinkParams p) {
    const double eps = ctl->eps, f0 = ctl->f0[0];
    double s = 0.0;
    for (int64_t j = static_cast<int64_t>(blockIdx.x) * 64 + threadIdx.x; j < nJ;
         j += static_cast<int64_t>(gridDim.x) * 64)
        s += exp((f0 + static_cast<double>(G[j]) - p.c_unm) / eps);
    s = wave_sum(s);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
    if (last_block(ctl)) {
        double t = 0.0;
        for (int w = threadIdx.x; w < static_cast<int>(gridDim.x); w += 64) t += part[w];
        t = wave_sum(t);
        if (threadIdx.x == 0) {
            ctl->cs_sum = t;
            ctl->ticket = 0u;
        }
    }
}

// ---------------------------------------------------------------- row pass

// Row half of Sinkhorn iteration k = iter + 1 for 64 detected spots of one
// block.  Each lane streams the block's model spots; with the previous f_i as
// shift every term is an entry of the current plan (<= 1 after a column
// half), so no running maximum is needed.  The sum S_i is the row marginal of
// state k-1 (its error is the convergence test) and f_i^k = f_i^{k-1} -
// eps ln S_i.  The last workgroup updates the bin potentials and decides
// convergence.
__global__ __launch_bounds__(64) void k_row(const Item *__restrict__ items,
                                            const float *__restrict__ P1,
                                            const float *__restrict__ P2,
                                            const Col8 *__restrict__ cols,
                                            const float *__restrict__ G, float *F0, float *F1,
                                            SinkCtl *ctl, double2 *__restrict__ part,
                                            SinkParams p) {
    if (ctl->done) return;
    const int k = ctl->iter + 1;
    const float *Fin = ((k - 1) & 1) ? F1 : F0;
    float *Fout = (k & 1) ? F1 : F0;
    const double eps = ctl->eps;
    const double kexp = ctl->kexp;
    const float kx = static_cast<float>(kexp);
    const float K = p.twoD2 * kx;
    const double g0 = ctl->g0[(k - 1) & 1];
    const Item it = items[blockIdx.x];
    const int i = it.r0 + static_cast<int>(threadIdx.x);
    const bool act = i < it.r1;
    const float p1 = act ? P1[i] : 0.0f;
    const float p2 = act ? P2[i] : 0.0f;
    const float f = act ? Fin[i] : 0.0f;
    const float fk = f * kx;
    double acc = 0.0;
    for (int j0 = it.c0; j0 < it.c1; j0 += 64) {
        const int j1 = min(j0 + 64, it.c1);
        float a = 0.0f;
#pragma unroll 4
        for (int j = j0; j < j1; ++j) {
            const Col8 c = cols[j];
            const float base = fmaf(G[j], kx, fk);
            a += fast_exp2(entry_exponent(p1, p2, c.s1, c.s2, c.v1, c.v2, c.vv, c.vv2, K, base));
        }
        acc += static_cast<double>(a);
    }
    const double eb = (g0 - p.c_out) * kexp + static_cast<double>(fk);
    acc += exp2(eb);
    double logS;
    const bool slow = act && !(acc > 1e-30);
    if (__any(slow)) {
        // every term underflowed: recompute with the row maximum as shift
        float mx = static_cast<float>(eb);
        for (int j = it.c0; j < it.c1; ++j) {
            const Col8 c = cols[j];
            mx = fmaxf(mx, entry_exponent(p1, p2, c.s1, c.s2, c.v1, c.v2, c.vv, c.vv2, K,
                                          fmaf(G[j], kx, fk)));
        }
        double s2 = exp2(eb - mx);
        for (int j = it.c0; j < it.c1; ++j) {
            const Col8 c = cols[j];
            s2 += exp2(static_cast<double>(entry_exponent(p1, p2, c.s1, c.s2, c.v1, c.v2, c.vv,
                                                          c.vv2, K, fmaf(G[j], kx, fk)) - mx));
        }
        logS = slow ? log(s2) + static_cast<double>(mx) * 0.6931471805599453 : log(acc);
    } else {
        logS = log(acc);
    }
    double err = act ? fabs(acc - 1.0) : 0.0;
    const double fn = static_cast<double>(f) - eps * logS;
    double rs = 0.0;
    if (act) {
        const float fnf = static_cast<float>(fn);
        Fout[i] = fnf;
        rs = exp((static_cast<double>(fnf) + g0 - p.c_out) / eps);
    }
    rs = wave_sum(rs);
    err = wave_max(err);
    if (threadIdx.x == 0) part[blockIdx.x] = make_double2(rs, err);
    if (!last_block(ctl)) return;
    double rsum = 0.0, emax = 0.0;
    for (int w = threadIdx.x; w < static_cast<int>(gridDim.x); w += 64) {
        rsum += part[w].x;
        emax = fmax(emax, part[w].y);
    }
    rsum = wave_sum(rsum);
    emax = wave_max(emax);
    if (threadIdx.x == 0) {
        const int slot = (k - 1) & 1;
        const double f0p = ctl->f0[slot], g0p = ctl->g0[slot];
        const double row0 = ctl->cs_sum + exp((f0p + g0p - p.c_sink) / eps);
        const double err0 = p.t_b > 0 ? fabs(row0 - p.t_b) / p.t_b : 0.0;
        const double e = fmax(emax, err0);
        if (e < 0.99 * ctl->best_err) {
            ctl->best_err = e;
            ctl->best_iter = k;
        }
        // FP32 potentials put a rounding floor under the marginal error (about
        // 1e-5 at the smallest temperatures): an error within 4 tol that has
        // not fallen by 1% over 64 iterations counts as converged
        const bool floor = e <= 4.0 * p.tol && k - ctl->best_iter >= 64;
        if (k >= 2 && (e <= p.tol || floor || k - 1 >= p.n_max)) {
            ctl->done = 1;
            ctl->final_state = k - 1;
            ctl->converged = (e <= p.tol || floor) ? 1 : 0;
            ctl->err = e;
        } else {
            const double f0n = p.t_b > 0 ? f0p + eps * log(p.t_b) - eps * log(row0) : -INFINITY;
            const double g0n =
                p.t_a > 0 ? g0p + eps * log(p.t_a) - eps * log(rsum + exp((f0n + g0p - p.c_sink) / eps))
                          : -INFINITY;
            ctl->f0[k & 1] = f0n;
            ctl->g0[k & 1] = g0n;
            ctl->iter = k;
            ctl->err = e;
        }
        ctl->ticket = 0u;
    }
}

// ---------------------------------------------------------------- column pass

// Column half of iteration k = iter for 64 model spots of one block: each
// lane streams the block's detected spots with g_j^{k-1} as shift (terms are
// entries of the plan after the row half, <= 1) and sets
// g_j^k = g_j^{k-1} - eps ln(column marginal).  The last workgroup stores
// sum_j exp((f0 + g_j - c_unm)/eps) for the next row half.
__global__ __launch_bounds__(64) void k_col(const Item *__restrict__ items,
                                            const float *__restrict__ P1,
                                            const float *__restrict__ P2,
                                            const Col8 *__restrict__ cols, float *G,
                                            const float *F0, const float *F1, SinkCtl *ctl,
                                            double2 *__restrict__ part, SinkParams p) {
    if (ctl->done) return;
    const int k = ctl->iter;
    const float *__restrict__ F = (k & 1) ? F1 : F0;
    const double eps = ctl->eps;
    const double kexp = ctl->kexp;
    const float kx = static_cast<float>(kexp);
    const float K = p.twoD2 * kx;
    const double f0 = ctl->f0[k & 1];
    const Item it = items[blockIdx.x];
    const int j = it.c0 + static_cast<int>(threadIdx.x);
    const bool act = j < it.c1;
    Col8 c = {0, 0, 0, 0, 1, 1, 1, 0};
    float g = 0.0f;
    if (act) {
        c = cols[j];
        g = G[j];
    }
    const float gk = g * kx;
    double acc = 0.0;
    for (int i0 = it.r0; i0 < it.r1; i0 += 64) {
        const int i1 = min(i0 + 64, it.r1);
        float a = 0.0f;
#pragma unroll 4
        for (int i = i0; i < i1; ++i) {
            const float base = fmaf(F[i], kx, gk);
            a += fast_exp2(entry_exponent(P1[i], P2[i], c.s1, c.s2, c.v1, c.v2, c.vv, c.vv2, K, base));
        }
        acc += static_cast<double>(a);
    }
    const double eb = (f0 - p.c_unm) * kexp + static_cast<double>(gk);
    acc += exp2(eb);
    double logS;
    const bool slow = act && !(acc > 1e-30);
    if (__any(slow)) {
        float mx = static_cast<float>(eb);
        for (int i = it.r0; i < it.r1; ++i)
            mx = fmaxf(mx, entry_exponent(P1[i], P2[i], c.s1, c.s2, c.v1, c.v2, c.vv, c.vv2, K,
                                          fmaf(F[i], kx, gk)));
        double s2 = exp2(eb - mx);
        for (int i = it.r0; i < it.r1; ++i)
            s2 += exp2(static_cast<double>(entry_exponent(P1[i], P2[i], c.s1, c.s2, c.v1, c.v2,
                                                          c.vv, c.vv2, K, fmaf(F[i], kx, gk))) -
                       mx);
        logS = slow ? log(s2) + static_cast<double>(mx) * 0.6931471805599453 : log(acc);
    } else {
        logS = log(acc);
    }
    double cs = 0.0;
    if (act) {
        const float gn = static_cast<float>(static_cast<double>(g) - eps * logS);
        G[j] = gn;
        cs = exp((f0 + static_cast<double>(gn) - p.c_unm) / eps);
    }
    cs = wave_sum(cs);
    if (threadIdx.x == 0) part[blockIdx.x] = make_double2(cs, 0.0);
    if (!last_block(ctl)) return;
    double t = 0.0;
    for (int w = threadIdx.x; w < static_cast<int>(gridDim.x); w += 64) t += part[w].x;
    t = wave_sum(t);
    if (threadIdx.x == 0) {
        ctl->cs_sum = t;
        ctl->ticket = 0u;
    }
}

// ---------------------------------------------------------------- plan / assign

// Hard assignment per detected spot: argmax_j Q_ij over its block and the
// outlier column (lowest index on ties, -1 = outlier).
__global__ __launch_bounds__(64) void k_assign(const Item *__restrict__ items,
                                               const float *__restrict__ P1,
                                               const float *__restrict__ P2,
                                               const Col8 *__restrict__ cols,
                                               const float *__restrict__ G,
                                               const float *__restrict__ F,
                                               const int *__restrict__ mgrain, double g0, double eps,
                                               SinkParams p, int *__restrict__ jstar,
                                               int *__restrict__ gstar, float *__restrict__ qstar,
                                               float *__restrict__ qout) {
    const Item it = items[blockIdx.x];
    const int i = it.r0 + static_cast<int>(threadIdx.x);
    const bool act = i < it.r1;
    const double kexp = 1.4426950408889634 / eps;
    const float kx = static_cast<float>(kexp);
    const float K = p.twoD2 * kx;
    const float p1 = act ? P1[i] : 0.0f, p2 = act ? P2[i] : 0.0f, f = act ? F[i] : 0.0f;
    const float fk = f * kx;
    float best = -INFINITY;
    int arg = -1;
    for (int j = it.c0; j < it.c1; ++j) {
        const Col8 c = cols[j];
        float e = entry_exponent(p1, p2, c.s1, c.s2, c.v1, c.v2, c.vv, c.vv2, K, fmaf(G[j], kx, fk));
        if (e > best) {
            best = e;
            arg = j;
        }
    }
    if (!act) return;
    const double eb = (g0 - p.c_out) * kexp + static_cast<double>(fk);
    const float qo = static_cast<float>(exp2(eb));
    const float qb = arg >= 0 ? fast_exp2(best) : 0.0f;
    if (jstar) jstar[i] = (arg >= 0 && qb >= qo) ? arg : -1;
    if (gstar) gstar[i] = (arg >= 0 && qb >= qo) ? mgrain[arg] : -1;
    if (qstar) qstar[i] = (arg >= 0 && qb >= qo) ? qb : qo;
    if (qout) qout[i] = qo;
}

// ---------------------------------------------------------------- M-step

// Per model spot (lane), stream the block's detected spots: the E-step plan
// weight Q_ij (from colsE) and the residual geometry at the current grains
// (colsC).  In the detector frame, with d = v + (p - s), tau = |d|,
// rhat = d / tau and P = I - rhat rhat^T, accumulate
//   S0 = sum Q, e = sum Q (rhat - r), A = sum Q P / tau^2, B = sum Q P / tau
// (rhat - r is formed as ((p - s) - r delta) / tau with
// delta = |d| - |v| = (2 v.(p-s) + |p-s|^2) / (|d| + |v|), free of
// cancellation).  The epilogue turns them into this column's FP64
// contribution to its grain's normal equations:
//   H_ww = D^2 S0 K^T K, H_xx = D^2 Gt^T A Gt, H_xw = D^2 Gt^T B K,
//   g_w = -D^2 K^T e,    g_x = D^2 Gt^T B r,
// with K = 2 (u e^T + (u.e) I) Gt [R w]_x the rotation Jacobian of the ray.
__global__ __launch_bounds__(64) void k_mstep_acc(
    const Item *__restrict__ items, const float *__restrict__ P1, const float *__restrict__ P2,
    const float *__restrict__ F, const float *__restrict__ G, const Col8 *__restrict__ colsE,
    const Col8 *__restrict__ colsC, const GeomF *__restrict__ Gp, const float *__restrict__ W,
    int n_planes, const GrainF *__restrict__ grains, int n_grains, const int *__restrict__ mplane,
    const int *__restrict__ mgrain, const int *__restrict__ mblock, float kx, float K, double D2,
    double *__restrict__ colHg) {
    const Item it = items[blockIdx.x];
    const int j = it.c0 + static_cast<int>(threadIdx.x);
    const bool act = j < it.c1;
    Col8 cE = {0, 0, 0, 0, 1, 1, 1, 0}, cC = {0, 0, 0, 0, 1, 1, 1, 0};
    float g = 0.0f;
    if (act) {
        cE = colsE[j];
        cC = colsC[j];
        g = G[j];
    }
    const float gk = g * kx;
    const float vlen = sqrtf(cC.vv);
    const float ivl = 1.0f / vlen;
    const float rn = cC.vn * ivl, r1 = cC.v1 * ivl, r2 = cC.v2 * ivl;
    double s64[kStat];
    for (int k = 0; k < kStat; ++k) s64[k] = 0.0;
    for (int i0 = it.r0; i0 < it.r1; i0 += 64) {
        const int i1 = min(i0 + 64, it.r1);
        float a[kStat];
        for (int k = 0; k < kStat; ++k) a[k] = 0.0f;
        for (int i = i0; i < i1; ++i) {
            const float p1 = P1[i], p2 = P2[i];
            const float Q = fast_exp2(entry_exponent(p1, p2, cE.s1, cE.s2, cE.v1, cE.v2, cE.vv,
                                                     cE.vv2, K, fmaf(F[i], kx, gk)));
            if (Q > 0.0f) accumulate_stats(a, Q, p1, p2, cC, vlen, rn, r1, r2);
        }
        for (int k = 0; k < kStat; ++k) s64[k] += static_cast<double>(a[k]);
    }
    if (!act) return;
    column_normal_equations(*Gp, W, n_planes, grains, n_grains, mplane[j], mgrain[j], mblock[j],
                            s64, rn, r1, r2, D2, colHg + static_cast<int64_t>(j) * kHg);
}

// One wave per grain: sum its columns' contributions (per block, the grain's
// columns are one contiguous run found by binary search), then lane 0 solves
// (H + mu I) step = -g by Cholesky in FP64 and applies the step.
__global__ __launch_bounds__(64) void k_mstep_solve(
    const double *__restrict__ colHg, const int *__restrict__ mgrain,
    const int64_t *__restrict__ mboff, int n_blocks, double mu_rel, double *q, double *x,
    GrainF *__restrict__ gf, double *__restrict__ step_norm) {
    const int n = blockIdx.x;
    double acc[kHg];
    for (int k = 0; k < kHg; ++k) acc[k] = 0.0;
    for (int b = threadIdx.x; b < n_blocks; b += 64) {
        int64_t lo = mboff[b], hi = mboff[b + 1];
        int64_t a = lo, e = hi;
        while (a < e) {
            int64_t mid = (a + e) >> 1;
            if (mgrain[mid] < n) a = mid + 1; else e = mid;
        }
        int64_t z = a;
        e = hi;
        while (z < e) {
            int64_t mid = (z + e) >> 1;
            if (mgrain[mid] <= n) z = mid + 1; else e = mid;
        }
        for (int64_t j = a; j < z; ++j)
            for (int k = 0; k < kHg; ++k) acc[k] += colHg[j * kHg + k];
    }
    for (int k = 0; k < kHg; ++k) acc[k] = wave_sum(acc[k]);
    if (threadIdx.x != 0) return;
    gn_solve_apply(acc, mu_rel, q + 4 * n, x + 3 * n, gf + n, step_norm ? step_norm + n : nullptr);
}

// ---------------------------------------------------------------- host side

struct Plan {
    std::vector<Item> rows, cols;
    int64_t entries = 0;   // sum_b I_b J_b
};

static Plan make_plan(const int64_t *ob, const int64_t *mb, int nb) {
    Plan p;
    for (int b = 0; b < nb; ++b) {
        int r0 = static_cast<int>(ob[b]), r1 = static_cast<int>(ob[b + 1]);
        int c0 = static_cast<int>(mb[b]), c1 = static_cast<int>(mb[b + 1]);
        p.entries += static_cast<int64_t>(r1 - r0) * (c1 - c0);
        for (int r = r0; r < r1; r += 64) p.rows.push_back({r, std::min(r + 64, r1), c0, c1});
        for (int c = c0; c < c1; c += 64) p.cols.push_back({r0, r1, c, std::min(c + 64, c1)});
    }
    // the passes always launch at least one (possibly empty) workgroup
    if (p.rows.empty()) p.rows.push_back({0, 0, 0, 0});
    if (p.cols.empty()) p.cols.push_back({0, 0, 0, 0});
    // heaviest items first so the tail of the grid is short
    std::stable_sort(p.rows.begin(), p.rows.end(),
                     [](const Item &a, const Item &b) { return (a.c1 - a.c0) > (b.c1 - b.c0); });
    std::stable_sort(p.cols.begin(), p.cols.end(),
                     [](const Item &a, const Item &b) { return (a.r1 - a.r0) > (b.r1 - b.r0); });
    return p;
}

static size_t n_items_max(int64_t n_obs, int64_t n_model, int nb) {
    return static_cast<size_t>((n_obs + 63) / 64 + (n_model + 63) / 64 + 2 * nb + 1);
}

struct EmWs {
    SinkCtl *ctl;
    double2 *part;
    Item *rows, *cols;
    float *F1;
    Col8 *colsE, *colsC;
    double *colHg;
    GeomF *geom;
    GrainF *grains;
    int64_t *mboff;
};

static size_t carve_em(Carver &cv, EmWs &w, const laue_geometry *g, int64_t n_obs, int64_t n_model,
                       int n_grains) {
    const int nb = g->n_rot * g->n_det;
    const size_t ni = n_items_max(n_obs, n_model, nb);
    w.ctl = cv.take<SinkCtl>(1);
    w.part = cv.take<double2>(ni);
    w.rows = cv.take<Item>(ni);
    w.cols = cv.take<Item>(ni);
    w.F1 = cv.take<float>(std::max<int64_t>(n_obs, 1));
    w.colsE = cv.take<Col8>(std::max<int64_t>(n_model, 1));
    w.colsC = cv.take<Col8>(std::max<int64_t>(n_model, 1));
    w.colHg = cv.take<double>(std::max<int64_t>(n_model, 1) * kHg);
    w.geom = cv.take<GeomF>(1);
    w.grains = cv.take<GrainF>(std::max(n_grains, 1));
    w.mboff = cv.take<int64_t>(nb + 1);
    return cv.size();
}

static int validate_obs(const laue_obs_spots *o, int nb) {
    LAUE_REQUIRE(o && o->block_off && o->n >= 0, LAUE_EINVAL, "detected spots or block_off is NULL");
    LAUE_REQUIRE(o->n == 0 || (o->p1 && o->p2), LAUE_EINVAL, "detected-spot arrays are NULL");
    LAUE_REQUIRE(o->block_off[0] == 0 && o->block_off[nb] == o->n, LAUE_EINVAL,
                 "detected-spot block offsets must run from 0 to n");
    for (int b = 0; b < nb; ++b)
        LAUE_REQUIRE(o->block_off[b + 1] >= o->block_off[b], LAUE_EINVAL,
                     "detected-spot block offsets must be non-decreasing");
    LAUE_REQUIRE(o->n < (int64_t(1) << 31), LAUE_EINVAL, "too many detected spots");
    return LAUE_OK;
}

static int validate_model(const laue_model_spots *m, int nb, bool need_geo) {
    LAUE_REQUIRE(m && m->block_off && m->n >= 0, LAUE_EINVAL, "model spots or block_off is NULL");
    LAUE_REQUIRE(m->n == 0 || (m->plane && m->grain && m->block), LAUE_EINVAL,
                 "model-spot id arrays are NULL");
    LAUE_REQUIRE(!need_geo || m->n == 0 || (m->s1 && m->s2 && m->vn && m->v1 && m->v2),
                 LAUE_EINVAL, "model-spot geometry arrays are NULL");
    LAUE_REQUIRE(m->block_off[0] == 0 && m->block_off[nb] == m->n, LAUE_EINVAL,
                 "model-spot block offsets must run from 0 to n");
    for (int b = 0; b < nb; ++b)
        LAUE_REQUIRE(m->block_off[b + 1] >= m->block_off[b], LAUE_EINVAL,
                     "model-spot block offsets must be non-decreasing");
    LAUE_REQUIRE(m->n < (int64_t(1) << 31), LAUE_EINVAL, "too many model spots");
    return LAUE_OK;
}

static int validate_ot(const laue_ot_params *p, bool need_eps) {
    LAUE_REQUIRE(p != nullptr, LAUE_EINVAL, "OT parameters are NULL");
    LAUE_REQUIRE(!need_eps || (std::isfinite(p->eps) && p->eps > 0), LAUE_EINVAL, "eps must be > 0");
    LAUE_REQUIRE(std::isfinite(p->distance) && p->distance > 0, LAUE_EINVAL, "distance must be > 0");
    LAUE_REQUIRE(std::isfinite(p->c_out) && std::isfinite(p->c_unm) && std::isfinite(p->c_sink),
                 LAUE_EINVAL, "bin costs must be finite");
    LAUE_REQUIRE(std::isfinite(p->t_b) && p->t_b >= 0, LAUE_EINVAL, "T_b must be >= 0");
    LAUE_REQUIRE(std::isfinite(p->tol) && p->tol >= 0, LAUE_EINVAL, "tol must be >= 0");
    LAUE_REQUIRE(p->n_max >= 1, LAUE_EINVAL, "n_max must be >= 1");
    return LAUE_OK;
}

// A prepared E/M-step problem on one stream.
struct Engine {
    hipStream_t s;
    EmWs w;
    Plan plan;
    SinkParams sp;
    const laue_obs_spots *obs;
    laue_model_spots *model;
    int nb;
    int64_t sink_entries = 0;
    // GPU time of the Sinkhorn passes and M-step passes (HIP events)
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    double sink_ms = 0.0, mstep_ms = 0.0;
    int64_t sink_passes = 0, sink_pass_entries = 0, mstep_entries = 0;

    ~Engine() {
        if (ev0) (void)hipEventDestroy(ev0);
        if (ev1) (void)hipEventDestroy(ev1);
    }

    int timer_start() {
        if (!ev0) {
            LAUE_CHECK_HIP(hipEventCreate(&ev0));
            LAUE_CHECK_HIP(hipEventCreate(&ev1));
        }
        LAUE_CHECK_HIP(hipEventRecord(ev0, s));
        return LAUE_OK;
    }

    int timer_stop(double *acc) {
        LAUE_CHECK_HIP(hipEventRecord(ev1, s));
        LAUE_CHECK_HIP(hipEventSynchronize(ev1));
        float ms = 0.0f;
        LAUE_CHECK_HIP(hipEventElapsedTime(&ms, ev0, ev1));
        *acc += ms;
        return LAUE_OK;
    }

    int upload(const laue_geometry *geom, const laue_ot_params *par) {
        plan = make_plan(obs->block_off, model->block_off, nb);
        std::vector<Item> rows = plan.rows, cols = plan.cols;
        if (!rows.empty())
            LAUE_CHECK_HIP(hipMemcpyAsync(w.rows, rows.data(), rows.size() * sizeof(Item),
                                          hipMemcpyHostToDevice, s));
        if (!cols.empty())
            LAUE_CHECK_HIP(hipMemcpyAsync(w.cols, cols.data(), cols.size() * sizeof(Item),
                                          hipMemcpyHostToDevice, s));
        LAUE_CHECK_HIP(hipMemcpyAsync(w.mboff, model->block_off, (nb + 1) * sizeof(int64_t),
                                      hipMemcpyHostToDevice, s));
        GeomF hg;
        make_geomf(geom, &hg);
        LAUE_CHECK_HIP(hipMemcpyAsync(w.geom, &hg, sizeof(GeomF), hipMemcpyHostToDevice, s));
        LAUE_CHECK_HIP(hipStreamSynchronize(s));
        sp.c_out = par->c_out;
        sp.c_unm = par->c_unm;
        sp.c_sink = par->c_sink;
        sp.t_b = par->t_b;
        sp.t_a = par->t_b + static_cast<double>(obs->n) - static_cast<double>(model->n);
        sp.tol = par->tol;
        sp.twoD2 = static_cast<float>(2.0 * par->distance * par->distance);
        sp.n_max = par->n_max;
        return LAUE_OK;
    }

    // Sinkhorn from (f, g, f0, g0) at temperature eps on the packed columns.
    int sinkhorn(double eps, int chunk, laue_potentials *pot, laue_ot_stats *st) {
        const int nrow = static_cast<int>(plan.rows.size());
        const int ncol = static_cast<int>(plan.cols.size());
        double g0_in = sp.t_a > 0 ? pot->g0 : -INFINITY;
        double f0_in = sp.t_b > 0 ? pot->f0 : -INFINITY;
        k_ctl_init<<<1, 1, 0, s>>>(w.ctl, f0_in, g0_in, eps);
        LAUE_CHECK_HIP(hipGetLastError());
        if (model->n > 0) {
            int nwg = static_cast<int>(std::min<int64_t>((model->n + 63) / 64, 1024));
            k_cs_init<<<nwg, 64, 0, s>>>(pot->g, model->n, w.ctl, reinterpret_cast<double *>(w.part), sp);
            LAUE_CHECK_HIP(hipGetLastError());
        }
        if (chunk <= 0) chunk = 16;
        SinkCtl h{};
        int launched = 0;
        for (;;) {
            int rc = timer_start();
            if (rc) return rc;
            for (int c = 0; c < chunk && launched < sp.n_max + 1; ++c, ++launched) {
                k_row<<<nrow, 64, 0, s>>>(w.rows, obs->p1, obs->p2, w.colsE, pot->g, pot->f,
                                          w.F1, w.ctl, w.part, sp);
                k_col<<<ncol, 64, 0, s>>>(w.cols, obs->p1, obs->p2, w.colsE, pot->g, pot->f,
                                          w.F1, w.ctl, w.part, sp);
            }
            LAUE_CHECK_HIP(hipGetLastError());
            if ((rc = timer_stop(&sink_ms))) return rc;
            LAUE_CHECK_HIP(hipMemcpyAsync(&h, w.ctl, sizeof(SinkCtl), hipMemcpyDeviceToHost, s));
            LAUE_CHECK_HIP(hipStreamSynchronize(s));
            if (h.done) break;
            if (launched >= sp.n_max + 1) {
                set_error("internal: Sinkhorn did not stop at its cap");
                return LAUE_EDEVICE;
            }
        }
        const int fin = h.final_state;
        if (fin & 1)
            LAUE_CHECK_HIP(hipMemcpyAsync(pot->f, w.F1, obs->n * sizeof(float),
                                          hipMemcpyDeviceToDevice, s));
        pot->f0 = h.f0[fin & 1];
        pot->g0 = h.g0[fin & 1];
        st->n_iter = fin;
        st->converged = h.converged;
        st->err = h.err;
        sink_entries += plan.entries * (2 * static_cast<int64_t>(fin) + 1);
        sink_passes += 2 * static_cast<int64_t>(fin) + 1;
        sink_pass_entries += plan.entries * (2 * static_cast<int64_t>(fin) + 1);
        return LAUE_OK;
    }

    // k_gn Gauss-Newton steps with the plan of (pot, eps, colsE) fixed.
    int mstep(const laue_planes *planes, laue_grains *grains, const laue_potentials *pot, double eps,
              double distance, const laue_gn_params *gn, double *step_norm) {
        const int ncol = static_cast<int>(plan.cols.size());
        const float kx = static_cast<float>(1.4426950408889634 / eps);
        const float K = sp.twoD2 * kx;
        int trc = timer_start();
        if (trc) return trc;
        for (int k = 0; k < gn->k_gn; ++k) {
            Col8 *cur = w.colsE;
            if (k > 0) {
                int rc = launch_eval(w.geom, planes, w.grains, grains->n, model->plane, model->grain,
                                     model->block, model->n, nullptr, nullptr, nullptr, nullptr,
                                     nullptr, nullptr, w.colsC, s);
                if (rc) return rc;
                cur = w.colsC;
            }
            if (model->n > 0) {
                k_mstep_acc<<<ncol, 64, 0, s>>>(w.cols, obs->p1, obs->p2, pot->f, pot->g, w.colsE,
                                                cur, w.geom, planes->w, planes->n, w.grains,
                                                grains->n, model->plane, model->grain,
                                                model->block, kx, K, distance * distance, w.colHg);
                LAUE_CHECK_HIP(hipGetLastError());
            }
            if (grains->n > 0) {
                k_mstep_solve<<<grains->n, 64, 0, s>>>(w.colHg, model->grain, w.mboff, nb,
                                                       gn->mu_rel, grains->q, grains->x, w.grains,
                                                       step_norm);
                LAUE_CHECK_HIP(hipGetLastError());
            }
            sink_entries += plan.entries;
            mstep_entries += plan.entries;
        }
        return timer_stop(&mstep_ms);
    }
};

static int setup_engine(Engine &e, const laue_geometry *geom, const laue_obs_spots *obs,
                        laue_model_spots *model, const laue_ot_params *par, int n_grains, void *ws,
                        size_t ws_bytes, void *stream, bool need_geo) {
    int rc;
    if ((rc = validate_geometry(geom))) return rc;
    e.nb = geom->n_rot * geom->n_det;
    if ((rc = validate_obs(obs, e.nb)) || (rc = validate_model(model, e.nb, need_geo))) return rc;
    double t_a = par->t_b + static_cast<double>(obs->n) - static_cast<double>(model->n);
    LAUE_REQUIRE(t_a >= 0, LAUE_EINFEASIBLE,
                 "infeasible masses: T_a = T_b + |I| - |J| = " + std::to_string(t_a) + " < 0");
    Carver cv(ws);
    size_t need = carve_em(cv, e.w, geom, obs->n, model->n, n_grains);
    if ((rc = check_ws(ws, ws_bytes, need))) return rc;
    e.s = static_cast<hipStream_t>(stream);
    e.obs = obs;
    e.model = model;
    return e.upload(geom, par);
}

}  // namespace laue

using namespace laue;

extern "C" size_t laue_sinkhorn_workspace_size(const laue_geometry *geom, int64_t n_obs,
                                               int64_t n_model, int32_t n_grains) {
    if (!geom || validate_geometry(geom) != LAUE_OK || n_obs < 0 || n_model < 0 || n_grains < 0)
        return 0;
    Carver cv(nullptr);
    EmWs w;
    return carve_em(cv, w, geom, n_obs, n_model, n_grains);
}

extern "C" int laue_sinkhorn(const laue_geometry *geom, const laue_obs_spots *obs,
                             const laue_model_spots *model, const laue_ot_params *par,
                             laue_potentials *pot, laue_ot_stats *stats, void *ws, size_t ws_bytes,
                             void *stream) {
    clear_error();
    int rc;
    if ((rc = validate_ot(par, true))) return rc;
    LAUE_REQUIRE(pot && stats, LAUE_EINVAL, "potentials or stats is NULL");
    LAUE_REQUIRE(std::isfinite(pot->f0) && std::isfinite(pot->g0), LAUE_EINVAL,
                 "bin potentials must be finite");
    Engine e;
    laue_model_spots *m = const_cast<laue_model_spots *>(model);
    if ((rc = setup_engine(e, geom, obs, m, par, 0, ws, ws_bytes, stream, true))) return rc;
    LAUE_REQUIRE(obs->n == 0 || pot->f, LAUE_EINVAL, "f is NULL");
    LAUE_REQUIRE(model->n == 0 || pot->g, LAUE_EINVAL, "g is NULL");
    if ((rc = launch_pack(model, e.w.colsE, e.s))) return rc;
    if ((rc = e.sinkhorn(par->eps, par->chunk, pot, stats))) return rc;
    LAUE_CHECK_HIP(hipStreamSynchronize(e.s));
    return stats->converged ? LAUE_OK : LAUE_ENOCONV;
}

__global__ void k_plan_soa(const float *__restrict__ P1, const float *__restrict__ P2,
                           const float *__restrict__ s1, const float *__restrict__ s2,
                           const float *__restrict__ vn, const float *__restrict__ v1,
                           const float *__restrict__ v2, const float *__restrict__ F,
                           const float *__restrict__ G, int r0, int nI, int c0, int nJ, float kx,
                           float K, float *__restrict__ Q) {
    int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= nI * nJ) return;
    int i = r0 + idx / nJ, j = c0 + idx % nJ;
    float vnn = vn[j];
    float vv = fmaf(v2[j], v2[j], fmaf(v1[j], v1[j], vnn * vnn));
    Q[idx] = fast_exp2(entry_exponent(P1[i], P2[i], s1[j], s2[j], v1[j], v2[j], vv, vv * vv, K,
                                      fmaf(F[i], kx, G[j] * kx)));
}

__global__ void k_cost_soa(const float *__restrict__ P1, const float *__restrict__ P2,
                           const float *__restrict__ s1, const float *__restrict__ s2,
                           const float *__restrict__ vn, const float *__restrict__ v1,
                           const float *__restrict__ v2, int r0, int nI, int c0, int nJ,
                           float twoD2, float *__restrict__ Cout) {
    int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= nI * nJ) return;
    int i = r0 + idx / nJ, j = c0 + idx % nJ;
    float vnn = vn[j];
    float vv = fmaf(v2[j], v2[j], fmaf(v1[j], v1[j], vnn * vnn));
    // entry_exponent(..., K = -1, base = 0) returns c' = c / (2 D^2)
    Cout[idx] = twoD2 * entry_exponent(P1[i], P2[i], s1[j], s2[j], v1[j], v2[j], vv, vv * vv,
                                       -1.0f, 0.0f);
}

extern "C" int laue_cost_block(const laue_geometry *geom, const laue_obs_spots *obs,
                               const laue_model_spots *model, double distance, int32_t block,
                               float *Cout, void *stream) {
    clear_error();
    int rc;
    if ((rc = validate_geometry(geom))) return rc;
    const int nb = geom->n_rot * geom->n_det;
    if ((rc = validate_obs(obs, nb)) || (rc = validate_model(model, nb, true))) return rc;
    LAUE_REQUIRE(block >= 0 && block < nb, LAUE_EINVAL, "block out of range");
    LAUE_REQUIRE(Cout != nullptr, LAUE_EINVAL, "output is NULL");
    LAUE_REQUIRE(std::isfinite(distance) && distance > 0, LAUE_EINVAL, "distance must be > 0");
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int r0 = static_cast<int>(obs->block_off[block]);
    const int nI = static_cast<int>(obs->block_off[block + 1]) - r0;
    const int c0 = static_cast<int>(model->block_off[block]);
    const int nJ = static_cast<int>(model->block_off[block + 1]) - c0;
    LAUE_REQUIRE(static_cast<int64_t>(nI) * nJ < (int64_t(1) << 31), LAUE_EINVAL, "block too large");
    if (nI == 0 || nJ == 0) return LAUE_OK;
    k_cost_soa<<<(nI * nJ + 255) / 256, 256, 0, s>>>(obs->p1, obs->p2, model->s1, model->s2,
                                                     model->vn, model->v1, model->v2, r0, nI, c0,
                                                     nJ, static_cast<float>(2.0 * distance * distance),
                                                     Cout);
    LAUE_CHECK_HIP(hipGetLastError());
    return LAUE_OK;
}

extern "C" int laue_plan_block(const laue_geometry *geom, const laue_obs_spots *obs,
                               const laue_model_spots *model, const laue_ot_params *par,
                               const laue_potentials *pot, int32_t block, float *Q, void *stream) {
    clear_error();
    int rc;
    if ((rc = validate_geometry(geom)) || (rc = validate_ot(par, true))) return rc;
    const int nb = geom->n_rot * geom->n_det;
    if ((rc = validate_obs(obs, nb)) || (rc = validate_model(model, nb, true))) return rc;
    LAUE_REQUIRE(block >= 0 && block < nb, LAUE_EINVAL, "block out of range");
    LAUE_REQUIRE(pot && pot->f && pot->g && Q, LAUE_EINVAL, "NULL argument");
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int r0 = static_cast<int>(obs->block_off[block]);
    const int nI = static_cast<int>(obs->block_off[block + 1]) - r0;
    const int c0 = static_cast<int>(model->block_off[block]);
    const int nJ = static_cast<int>(model->block_off[block + 1]) - c0;
    LAUE_REQUIRE(static_cast<int64_t>(nI) * nJ < (int64_t(1) << 31), LAUE_EINVAL, "block too large");
    if (nI == 0 || nJ == 0) return LAUE_OK;
    const float kx = static_cast<float>(1.4426950408889634 / par->eps);
    const float K = static_cast<float>(2.0 * par->distance * par->distance) * kx;
    k_plan_soa<<<(nI * nJ + 255) / 256, 256, 0, s>>>(obs->p1, obs->p2, model->s1, model->s2,
                                                     model->vn, model->v1, model->v2, pot->f,
                                                     pot->g, r0, nI, c0, nJ, kx, K, Q);
    LAUE_CHECK_HIP(hipGetLastError());
    return LAUE_OK;
}

extern "C" int laue_mstep(const laue_geometry *geom, const laue_planes *planes,
                          const laue_obs_spots *obs, laue_model_spots *model,
                          const laue_ot_params *par, const laue_potentials *pot,
                          const laue_gn_params *gn, laue_grains *grains, double *step_norm,
                          void *ws, size_t ws_bytes, void *stream) {
    clear_error();
    int rc;
    if ((rc = validate_ot(par, true)) || (rc = validate_planes(planes)) || (rc = validate_grains(grains)))
        return rc;
    LAUE_REQUIRE(gn && gn->k_gn >= 0 && std::isfinite(gn->mu_rel) && gn->mu_rel >= 0, LAUE_EINVAL,
                 "bad Gauss-Newton parameters");
    LAUE_REQUIRE(pot && (obs == nullptr || obs->n == 0 || pot->f) && (model->n == 0 || pot->g),
                 LAUE_EINVAL, "potentials are NULL");
    Engine e;
    if ((rc = setup_engine(e, geom, obs, model, par, grains->n, ws, ws_bytes, stream, true))) return rc;
    if ((rc = launch_pack(model, e.w.colsE, e.s))) return rc;
    if ((rc = prep_grains(grains, e.w.grains, e.s))) return rc;
    if ((rc = e.mstep(planes, grains, pot, par->eps, par->distance, gn, step_norm))) return rc;
    LAUE_CHECK_HIP(hipStreamSynchronize(e.s));
    return LAUE_OK;
}

extern "C" int laue_em(const laue_geometry *geom, const laue_planes *planes,
                       const laue_obs_spots *obs, laue_model_spots *model,
                       const laue_em_params *par, laue_grains *grains, laue_potentials *pot,
                       laue_assignments *assign, laue_em_stats *stats, void *ws, size_t ws_bytes,
                       void *stream) {
    clear_error();
    int rc;
    LAUE_REQUIRE(par && stats && pot, LAUE_EINVAL, "NULL argument");
    if ((rc = validate_ot(&par->ot, false)) || (rc = validate_planes(planes)) ||
        (rc = validate_grains(grains)))
        return rc;
    LAUE_REQUIRE(par->n_stages >= 1 && par->iters_per_stage >= 1 && std::isfinite(par->eps_start) &&
                     std::isfinite(par->eps_end) && par->eps_start > 0 && par->eps_end > 0,
                 LAUE_EINVAL, "bad temperature schedule");
    LAUE_REQUIRE(par->gn.k_gn >= 0 && std::isfinite(par->gn.mu_rel) && par->gn.mu_rel >= 0,
                 LAUE_EINVAL, "bad Gauss-Newton parameters");
    LAUE_REQUIRE(std::isfinite(pot->f0) && std::isfinite(pot->g0), LAUE_EINVAL,
                 "bin potentials must be finite");
    Engine e;
    if ((rc = setup_engine(e, geom, obs, model, &par->ot, grains->n, ws, ws_bytes, stream, false)))
        return rc;
    LAUE_REQUIRE(obs->n == 0 || pot->f, LAUE_EINVAL, "f is NULL");
    LAUE_REQUIRE(model->n == 0 || pot->g, LAUE_EINVAL, "g is NULL");
    if ((rc = prep_grains(grains, e.w.grains, e.s))) return rc;
    *stats = laue_em_stats{};
    const int S = par->n_stages;
    for (int st = 0; st < S; ++st) {
        const double eps = S == 1 ? par->eps_start
                                  : par->eps_start * std::pow(par->eps_end / par->eps_start,
                                                              static_cast<double>(st) / (S - 1));
        for (int it = 0; it < par->iters_per_stage; ++it) {
            rc = launch_eval(e.w.geom, planes, e.w.grains, grains->n, model->plane, model->grain, model->block,
                             model->n, model->s1, model->s2, model->vn, model->v1, model->v2,
                             model->lam, e.w.colsE, e.s);
            if (rc) return rc;
            laue_ot_stats os{};
            if ((rc = e.sinkhorn(eps, par->ot.chunk, pot, &os))) return rc;
            stats->sinkhorn_iters += os.n_iter;
            stats->not_converged += os.converged ? 0 : 1;
            stats->last_err = os.err;
            if ((rc = e.mstep(planes, grains, pot, eps, par->ot.distance, &par->gn, nullptr))) return rc;
            stats->n_em_iter += 1;
        }
    }
    if (assign && obs->n > 0) {
        // assignments at the final grains with the final potentials
        const double eps_fin = par->eps_end;
        int rc2 = launch_eval(e.w.geom, planes, e.w.grains, grains->n, model->plane, model->grain, model->block,
                              model->n, model->s1, model->s2, model->vn, model->v1, model->v2,
                              model->lam, e.w.colsE, e.s);
        if (rc2) return rc2;
        k_assign<<<static_cast<int>(e.plan.rows.size()), 64, 0, e.s>>>(
            e.w.rows, obs->p1, obs->p2, e.w.colsE, pot->g, pot->f, model->grain, pot->g0,
            S == 1 ? par->eps_start : eps_fin, e.sp, assign->j_star, assign->grain,
            assign->q_star, assign->q_out);
        LAUE_CHECK_HIP(hipGetLastError());
        e.sink_entries += e.plan.entries;
    }
    stats->cost_entries = e.sink_entries;
    stats->sinkhorn_ms = e.sink_ms;
    stats->sinkhorn_passes = e.sink_passes;
    stats->sinkhorn_entries = e.sink_pass_entries;
    stats->mstep_ms = e.mstep_ms;
    stats->mstep_entries = e.mstep_entries;
    LAUE_CHECK_HIP(hipStreamSynchronize(e.s));
    return stats->not_converged ? LAUE_ENOCONV : LAUE_OK;
}
