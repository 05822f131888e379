// E-step (streamed log-domain Sinkhorn with outlier row/column), M-step
// (per-grain weighted Gauss-Newton) and the EM driver, for one sample or a
// batch of independent samples.
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
// other side of that block through LDS, 64 spots at a time (each lane loads
// one, every lane then reads each one by a broadcast LDS load, so the entry
// arithmetic has vector-register operands only), so the |I_b| x |J_b| cost
// block is recomputed on the fly and never stored.
//
// Batching: every sample has a descriptor (its arrays, bins, temperature and
// control block); a work item names its sample and its index within that
// sample.  One launch per pass covers all samples; each sample finalises its
// own bins in the last of its workgroups (a per-sample ticket) and stops on
// its own; workgroups of finished samples exit at once.  A sample's
// arithmetic does not depend on the other samples in the batch.
#include <algorithm>
#include <array>
#include <mutex>
#include <cmath>
#include <numeric>
#include <vector>

#include <hipcub/hipcub.hpp>

#include "common.h"

namespace laue {

int launch_pack(const laue_model_spots *m, Col8 *cols, hipStream_t s);

struct Item {
    int r0, r1, c0, c1;
    int s;        // sample
    int local;    // index among the sample's items of this pass
    int pad[2];
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
    double errf, errg;     // unbalanced / partial OT: largest marginal change of the latest row / column half
    double H;              // partial OT: mass potential (Q = exp((f + g + H - c) / eps))
};

struct SinkParams {
    double c_out, c_unm, c_sink, t_a, t_b, tol;
    double kappa, lam;     // unbalanced OT: marginal penalties (unb = 1)
    double mass;           // partial OT: transported mass m (part = 1)
    float twoD2;
    int n_max;
    int unb;               // 1: unbalanced OT (no bins)
    int part;              // 1: partial OT (no bins)
};

// New potential of a row (column) from ln S, S the sum of the previous
// state's plan entries of that row (column) including its bin entry.  The
// paper's model: u - eps ln S (Alg. BalancedOT).  Unbalanced OT (Alg.
// UnbalancedOT): tau (u - eps ln S), tau = kappa / (kappa + eps) for rows and
// lam / (lam + eps) for columns, and 0 for a row (column) without entries.
__device__ __forceinline__ float potential_update(float u, double logS, double eps, bool unb, double tau,
                                                  bool empty) {
    if (!unb) return static_cast<float>(static_cast<double>(u) - eps * logS);
    return empty ? 0.0f : static_cast<float>(tau * (static_cast<double>(u) - eps * logS));
}

// Partial OT (Alg. PartialOT, Dykstra's projections from the Gibbs kernel in
// potential form): here S sums exp((v + H - c)/eps) over the row (column),
// v the other side's potentials, and the new potential is min(0, -eps ln S)
// (0 without entries).  The stopping value is the change of the row's
// (column's) plan mass exp(ln S + u/eps) from the previous iteration's (prev;
// none in the first); the new mass is stored in prev.
__device__ __forceinline__ float partial_update(double logS, double eps, bool empty) {
    return empty ? 0.0f : static_cast<float>(fmin(0.0, -eps * logS));
}
__device__ __forceinline__ double partial_change(double logS, float u, double eps, bool empty, int k, float *prev) {
    const double m = empty ? 0.0 : exp(logS + static_cast<double>(u) / eps);
    const double d = k > 1 ? fabs(m - static_cast<double>(*prev)) : INFINITY;
    *prev = static_cast<float>(m);
    return d;
}

// Unbalanced OT's stopping value for one row (column): the change its update
// makes to its plan marginal, S |exp((u_new - u)/eps) - 1| with S = exp(logS)
// the mass before the update (0 for a row without entries).
__device__ __forceinline__ double mass_change(double logS, float u_new, float u, double eps, bool empty) {
    if (empty) return 0.0;
    const double d = (static_cast<double>(u_new) - static_cast<double>(u)) / eps;
    return fabs(exp(logS + d) - exp(logS));
}

// Everything a kernel needs about one sample.
struct SampleDesc {
    const float *p1, *p2;          // detected spots
    float *f, *f1, *g;             // potentials (f1: odd states, ws)
    Col8 *colsE, *colsC;           // packed columns: plan geometry / current geometry
    SinkCtl *ctl;
    double2 *part;                 // per-item partials of a pass
    int n_row_items, n_col_items;  // 64-row / 64-column items
    int n_row_wg2, n_col_wg2;      // workgroups of the two-per-lane tile shape
    SinkParams sp;
    const int *mplane, *mgrain, *mblock;
    float *s1, *s2, *vn, *v1, *v2, *lam;   // forward-model outputs (may be NULL)
    const int64_t *mboff;          // model-spot block offsets (device)
    int64_t n_obs, n_model;
    int nb, n_grains, n_planes, pad0;
    const GeomF *geom;
    GrainF *grains;
    double *q, *x;
    double *colHg;
    double *step_norm;             // may be NULL
    const float *W, *Dsp;
    double D2, mu_rel;
    int *jstar, *gstar;            // assignments (may be NULL)
    float *qstar, *qout;
    // sparse assignment (rho > 0): neighbour sets and their column lists
    int rho, cand_cap;             // neighbours per detected spot; filter capacity per row
    float knn_k;                   // filter threshold = knn_k / (model spots of the block)
    int *nbr;                      // [n_obs x rho]
    int *nbr_prev;                 // [n_obs x rho] the previous E-step's (plan change)
    float *ncp;                    // [n_obs x rho] c / (2 D^2)
    int *cand_j, *cand_n;          // [n_obs x cand_cap], [n_obs]
    float *cand_c;                 // [n_obs x cand_cap]
    int *knn_list, *knn_nlist;     // rows for the exact pass
    int64_t *col_off;              // [n_model + 1]
    int *col_row;                  // [n_obs x rho]
    float *col_cp;                 // [n_obs x rho]
    const int64_t *oboff;          // detected-spot block offsets (device)
    int *knn_hist;                 // [nb x kGrid^2] model spots per detector cell
    int *sort_key, *sort_val;      // [n_obs x rho] radix-sort input (column, entry)
    const int *sorted_val;         // [n_obs x rho] entries ordered by column
    // partial OT: plan masses of the previous iteration (stopping test)
    float *rmass, *cmass;          // [n_obs], [n_model]
    // the paper's coordinate-descent M-step
    int *gflag;                    // [n_grains] Newton converged in this sweep
    int k_mm, pad1;                // MM steps per sweep
    double tol_x, tol_r;           // Newton and MM stops
    // plan summaries and the plan change between EM iterations
    double *obj;                   // [4 * (row items + column items) + 8] partials and totals
    float *qunm;                   // [n_model] Q_0j of the assignment output (may be NULL)
    Col8 *colsP;                   // previous E-step's packed columns
    float *fprev, *gprev;          // previous E-step's potentials
};

// ---------------------------------------------------------------- helpers

__device__ __forceinline__ bool last_block(SinkCtl *ctl, int n_items) {
    __shared__ int is_last;
    __threadfence();
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned t = atomicAdd(&ctl->ticket, 1u);
        is_last = (t == static_cast<unsigned>(n_items) - 1u) ? 1 : 0;
    }
    __syncthreads();
    if (is_last) __threadfence();
    return is_last != 0;
}

// Pointers read from a descriptor are generic; the pass bodies take the hot
// arrays as global-address-space, restrict-qualified parameters.
#define LAUE_GLOBAL __attribute__((address_space(1)))
template <class T>
__device__ __forceinline__ LAUE_GLOBAL T *gptr(T *p) {
    return (LAUE_GLOBAL T *)p;
}

__device__ __forceinline__ Col8 ld_col(const LAUE_GLOBAL Col8 *p) {
    return Col8{p->s1, p->s2, p->v1, p->v2, p->vv, p->vv2, p->vn, p->pad};
}

// sample s with base[s] <= i < base[s + 1] (base non-decreasing, n + 1 entries)
__device__ __forceinline__ int sample_of(const int64_t *base, int n, int64_t i) {
    int lo = 0, hi = n;
    while (hi - lo > 1) {
        const int mid = (lo + hi) / 2;
        if (base[mid] <= i) lo = mid; else hi = mid;
    }
    return lo;
}

struct CtlInit {
    double f0, g0, eps;
    double shift;          // gauge shift C of the solve's start state (f -= C, g += C)
};

// A plan Q = exp((f + g - c)/eps) of one sample for the summary and
// plan-change passes: its temperature and bin potentials (f, g and the
// columns come from the descriptor).
struct ObjIn {
    double eps, f0, g0;
};

__global__ void k_ctl_init(const SampleDesc *__restrict__ descs, int n, const CtlInit *__restrict__ init) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    SinkCtl *ctl = descs[s].ctl;
    const CtlInit v = init[s];
    ctl->f0[0] = v.f0;
    ctl->g0[0] = v.g0;
    ctl->f0[1] = v.f0;
    ctl->g0[1] = v.g0;
    ctl->cs_sum = 0.0;
    ctl->err = INFINITY;
    ctl->eps = v.eps;
    ctl->kexp = 1.4426950408889634 / v.eps;
    ctl->iter = 0;
    ctl->done = 0;
    ctl->best_iter = 0;
    ctl->best_err = INFINITY;
    ctl->errf = INFINITY;
    ctl->errg = INFINITY;
    ctl->H = 0.0;
    ctl->final_state = 0;
    ctl->converged = 0;
    ctl->ticket = 0u;
}

// Gauge of a warm start (outlier row and column only): the plan depends on
// the potentials only through f_i + g_j, f_i + g0, f0 + g_j and f0 + g0, so
// (f - C, g + C, f0 - C, g0 + C) is the same state.  Solves start from C = f0
// (f0 = 0 after the shift): a warm start carried down the temperatures
// otherwise keeps the common offset of its first, hot solve (|f|, |g| near
// 270 mm^2 at 1000 grains), and FP32 potentials of that size round each plan
// exponent by about 1.5e-5 at eps = 1.1 mm^2, a floor above the marginal
// tolerance.  One block row per sample (blockIdx.y).
__global__ void k_gauge(const SampleDesc *__restrict__ descs, const CtlInit *__restrict__ init) {
    const SampleDesc &D = descs[blockIdx.y];
    const double C = init[blockIdx.y].shift;
    if (C == 0.0) return;
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < D.n_obs) D.f[i] = static_cast<float>(static_cast<double>(D.f[i]) - C);
    if (i < D.n_model) D.g[i] = static_cast<float>(static_cast<double>(D.g[i]) + C);
}

// cs_sum of the initial state: sum_j exp((f0 + g_j - c_unm)/eps).  One wave
// per column item (up to 64 model spots) writes the item's partial; then one
// wave per sample sums them in item order (fixed summation order, no
// cross-wave atomics).
__global__ __launch_bounds__(64) void k_cs_init(const Item *__restrict__ items,
                                                const SampleDesc *__restrict__ descs) {
    const Item it = items[blockIdx.x];
    const SampleDesc &D = descs[it.s];
    const SinkCtl *ctl = D.ctl;
    const double eps = ctl->eps, f0 = ctl->f0[0];
    const int j = it.c0 + static_cast<int>(threadIdx.x);
    double s = j < it.c1 ? exp((f0 + static_cast<double>(D.g[j]) - D.sp.c_unm) / eps) : 0.0;
    s = wave_sum(s);
    if (threadIdx.x == 0) D.part[it.local] = make_double2(s, 0.0);
}

__global__ __launch_bounds__(256) void k_cs_final(const SampleDesc *__restrict__ descs) {
    const SampleDesc &D = descs[blockIdx.x];
    __shared__ double ws[4];
    double t = 0.0;
    for (int w = threadIdx.x; w < D.n_col_items; w += 256) t += D.part[w].x;
    t = wave_sum(t);
    if ((threadIdx.x & 63) == 0) ws[threadIdx.x >> 6] = t;
    __syncthreads();
    if (threadIdx.x == 0) D.ctl->cs_sum = ((ws[0] + ws[1]) + ws[2]) + ws[3];
}

// ---------------------------------------------------------------- row pass

// The sample's last workgroup of a row half: sums the item partials in item
// order, updates the bin potentials f0, g0 and decides convergence.
__device__ __forceinline__ void row_finalize(SinkCtl *__restrict__ ctl, const double2 *__restrict__ part,
                                             const SinkParams &p, int n_items, int k, double eps) {
    double rsum = 0.0, emax = 0.0;
    for (int w = threadIdx.x; w < n_items; w += 64) {
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
        double e = fmax(emax, err0);
        if (p.unb || p.part) {
            // unbalanced / partial OT: the marginal changes of iteration k-1 decide
            // whether state k-1 is final; this half's changes wait for the next
            e = fmax(ctl->errf, ctl->errg);
            ctl->errf = emax;
        }
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

// The sample's last workgroup of a column half: stores
// sum_j exp((f0 + g_j - c_unm)/eps) for the next row half and the largest
// marginal change of the half (unbalanced and partial OT's stopping test);
// under partial OT it applies the mass step.
__device__ __forceinline__ void col_finalize(SinkCtl *__restrict__ ctl, const double2 *__restrict__ part,
                                             int n_items, const SinkParams &p) {
    double t = 0.0, m = 0.0;
    for (int w = threadIdx.x; w < n_items; w += 64) {
        t += part[w].x;
        m = fmax(m, part[w].y);
    }
    t = wave_sum(t);
    m = wave_max(m);
    if (threadIdx.x == 0) {
        ctl->cs_sum = t;
        ctl->errg = m;
        // partial OT: the partials hold min(1, column sum) (the mass after the
        // column step); scale the plan to the mass m
        if (p.part && t > 0.0) ctl->H += ctl->eps * log(p.mass / t);
        ctl->ticket = 0u;
    }
}



// Row half of Sinkhorn iteration k = iter + 1 for 64 detected spots of one
// block.  Each lane streams the block's model spots; with the previous f_i as
// shift every term is an entry of the current plan (<= 1 after a column
// half), so no running maximum is needed.  The sum S_i is the row marginal of
// state k-1 (its error is the convergence test) and f_i^k = f_i^{k-1} -
// eps ln S_i.  The sample's last workgroup updates its bin potentials and
// decides its convergence.
// The block's columns come through LDS in chunks of 64 (double-buffered, the
// next chunk's global loads in flight while a chunk is summed).
// Tile shapes: R = 1 (one detected spot per lane, 64-row workgroups) or
// R = 2 (two adjacent 64-row items of one block per workgroup, two rows per
// lane sharing every column read).  Each 64-row item keeps its own partial and
// per-row arithmetic, so both shapes give identical results; the sample's
// ticket counts the workgroups of the launched shape (n_wg), its finalisation
// sums the partials of all 64-row items (n_items).
template <int R>
__device__ __forceinline__ void row_pass(const Item *its, const LAUE_GLOBAL float *__restrict__ P1,
                                         const LAUE_GLOBAL float *__restrict__ P2,
                                         const LAUE_GLOBAL Col8 *__restrict__ cols,
                                         const LAUE_GLOBAL float *__restrict__ G, LAUE_GLOBAL float *__restrict__ F0,
                                         LAUE_GLOBAL float *__restrict__ F1, SinkCtl *__restrict__ ctl,
                                         double2 *__restrict__ part, const SinkParams &p, int n_wg, int n_items,
                                         float *__restrict__ RM) {
    if (ctl->done) return;
    const int k = ctl->iter + 1;
    const LAUE_GLOBAL float *Fin = ((k - 1) & 1) ? F1 : F0;
    LAUE_GLOBAL float *Fout = (k & 1) ? F1 : F0;
    const double eps = ctl->eps;
    const double kexp = ctl->kexp;
    const float kx = static_cast<float>(kexp);
    const float K = p.twoD2 * kx;
    const double g0 = ctl->g0[(k - 1) & 1];
    const int c0 = its[0].c0, c1 = its[0].c1;
    int i[R];
    bool act[R];
    float p1[R], p2[R], f[R], fk[R];
    double acc[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        i[r] = its[r].r0 + static_cast<int>(threadIdx.x);
        act[r] = i[r] < its[r].r1;
        p1[r] = act[r] ? P1[i[r]] : 0.0f;
        p2[r] = act[r] ? P2[i[r]] : 0.0f;
        f[r] = act[r] ? Fin[i[r]] : 0.0f;
        // partial OT: the row sums of the Dykstra-corrected plan take the mass potential as shift
        fk[r] = p.part ? static_cast<float>(ctl->H * kexp) : f[r] * kx;
        acc[r] = 0.0;
    }
    {
        // 64 columns at a time through LDS (lane t loads column j0 + t, the
        // next chunk's load in flight while this one is summed); every lane
        // then reads each column by a broadcast LDS load, so the entry
        // arithmetic takes vector-register operands only
        __shared__ float4 lc[2][64][2];
        const int lane = static_cast<int>(threadIdx.x);
        float4 na = make_float4(0.0f, 0.0f, 0.0f, 0.0f), nb = na;
        if (c0 + lane < c1) {
            const Col8 c = ld_col(cols + c0 + lane);
            na = make_float4(c.s1, c.s2, c.v1, c.v2);
            nb = make_float4(c.vv, c.vv2, G[c0 + lane], 0.0f);
        }
        int buf = 0;
        for (int j0 = c0; j0 < c1; j0 += 64) {
            const int nj = min(64, c1 - j0);
            lc[buf][lane][0] = na;
            lc[buf][lane][1] = nb;
            __syncthreads();
            const int jn = j0 + 64 + lane;
            if (jn < c1) {
                const Col8 c = ld_col(cols + jn);
                na = make_float4(c.s1, c.s2, c.v1, c.v2);
                nb = make_float4(c.vv, c.vv2, G[jn], 0.0f);
            }
            float a[R];
#pragma unroll
            for (int r = 0; r < R; ++r) a[r] = 0.0f;
#pragma unroll 4
            for (int t = 0; t < nj; ++t) {
                const float4 A = lc[buf][t][0], B = lc[buf][t][1];
#pragma unroll
                for (int r = 0; r < R; ++r)
                    a[r] += fast_exp2(entry_exponent(p1[r], p2[r], A.x, A.y, A.z, A.w, B.x, B.y, K,
                                                     fmaf(B.z, kx, fk[r])));
            }
#pragma unroll
            for (int r = 0; r < R; ++r) acc[r] += static_cast<double>(a[r]);
            buf ^= 1;
        }
    }
    double eb[R], logS[R];
    bool slow[R], any_slow = false;
#pragma unroll
    for (int r = 0; r < R; ++r) {
        eb[r] = (g0 - p.c_out) * kexp + static_cast<double>(fk[r]);
        acc[r] += exp2(eb[r]);
        slow[r] = act[r] && !(acc[r] > 1e-30 && acc[r] < 1e30);
        any_slow = any_slow || slow[r];
        logS[r] = log(acc[r]);
    }
    if (__any(any_slow)) {
        // every term underflowed (or, under partial OT, the sum overflowed):
        // recompute with the row maximum as shift
#pragma unroll
        for (int r = 0; r < R; ++r) {
            float mx = static_cast<float>(eb[r]);
            for (int j = c0; j < c1; ++j) {
                const Col8 c = ld_col(cols + j);
                mx = fmaxf(mx, entry_exponent(p1[r], p2[r], c.s1, c.s2, c.v1, c.v2, c.vv, c.vv2, K,
                                              fmaf(G[j], kx, fk[r])));
            }
            double s2 = exp2(eb[r] - mx);
            for (int j = c0; j < c1; ++j) {
                const Col8 c = ld_col(cols + j);
                s2 += exp2(static_cast<double>(entry_exponent(p1[r], p2[r], c.s1, c.s2, c.v1, c.v2, c.vv,
                                                              c.vv2, K, fmaf(G[j], kx, fk[r])) - mx));
            }
            if (slow[r]) logS[r] = log(s2) + static_cast<double>(mx) * 0.6931471805599453;
        }
    }
    const bool unb = p.unb != 0;
    const double tau = unb ? p.kappa / (p.kappa + eps) : 1.0;
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const float fnf = p.part ? partial_update(logS[r], eps, c1 <= c0)
                                 : potential_update(f[r], logS[r], eps, unb, tau, c1 <= c0);
        double err = !act[r] ? 0.0
                     : p.part ? partial_change(logS[r], f[r], eps, c1 <= c0, k, RM + i[r])
                     : unb    ? mass_change(logS[r], fnf, f[r], eps, c1 <= c0)
                              : fabs(acc[r] - 1.0);
        double rs = 0.0;
        if (act[r]) {
            Fout[i[r]] = fnf;
            rs = exp((static_cast<double>(fnf) + g0 - p.c_out) / eps);
        }
        rs = wave_sum(rs);
        err = wave_max(err);
        if (threadIdx.x == 0 && its[r].local >= 0) part[its[r].local] = make_double2(rs, err);
    }
    if (!last_block(ctl, n_wg)) return;
    row_finalize(ctl, part, p, n_items, k, eps);
}

// the items of one workgroup of shape R: groups[w] = (first item, second item or -1)
template <int R>
__device__ __forceinline__ void group_items(const Item *__restrict__ items, const int2 *__restrict__ groups,
                                            Item *its) {
    if constexpr (R == 1) {
        its[0] = items[blockIdx.x];
    } else {
        const int2 gp = groups[blockIdx.x];
        its[0] = items[gp.x];
        its[R - 1] = gp.y >= 0 ? items[gp.y] : Item{0, 0, 0, 0, its[0].s, -1, {0, 0}};
    }
}

template <int R>
__global__ __launch_bounds__(64) void k_row(const Item *__restrict__ items, const int2 *__restrict__ groups,
                                            const SampleDesc *__restrict__ descs) {
    Item its[R];
    group_items<R>(items, groups, its);
    const SampleDesc &D = descs[its[0].s];
    row_pass<R>(its, gptr(D.p1), gptr(D.p2), gptr(D.colsE), gptr(D.g), gptr(D.f), gptr(D.f1), D.ctl, D.part,
                D.sp, R == 1 ? D.n_row_items : D.n_row_wg2, D.n_row_items, D.rmass);
}

// ---------------------------------------------------------------- column pass

// Column half of iteration k = iter for 64 model spots of one block (R = 2:
// two adjacent 64-column items per workgroup, two columns per lane sharing
// every row read): each lane streams the block's detected spots (through
// LDS, 64 at a time) with
// g_j^{k-1} as shift (terms are entries of the plan after the row half, <= 1)
// and sets g_j^k = g_j^{k-1} - eps ln(column marginal).  The sample's last
// workgroup stores sum_j exp((f0 + g_j - c_unm)/eps) for the next row half.
// Column sums of R adjacent 64-column items over the block's rows (p1, p2 and
// the row potentials F staged through LDS).
template <int R>
__device__ __forceinline__ void col_sums(const LAUE_GLOBAL float *__restrict__ P1,
                                         const LAUE_GLOBAL float *__restrict__ P2,
                                         const LAUE_GLOBAL float *__restrict__ F, int r0, int r1, const Col8 *c,
                                         const float *gk, float K, float kx, double *acc) {
    // 64 rows at a time through LDS (p1, p2, f of row i0 + lane), read back
    // by broadcast LDS loads: vector-register operands only
    __shared__ float4 lr[2][64];
    const int lane = static_cast<int>(threadIdx.x);
    float4 nx = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    if (r0 + lane < r1) nx = make_float4(P1[r0 + lane], P2[r0 + lane], F[r0 + lane], 0.0f);
    int buf = 0;
    for (int i0 = r0; i0 < r1; i0 += 64) {
        const int ni = min(64, r1 - i0);
        lr[buf][lane] = nx;
        __syncthreads();
        const int in = i0 + 64 + lane;
        if (in < r1) nx = make_float4(P1[in], P2[in], F[in], 0.0f);
        float a[R];
#pragma unroll
        for (int r = 0; r < R; ++r) a[r] = 0.0f;
#pragma unroll 4
        for (int t = 0; t < ni; ++t) {
            const float4 X = lr[buf][t];
#pragma unroll
            for (int r = 0; r < R; ++r)
                a[r] += fast_exp2(entry_exponent(X.x, X.y, c[r].s1, c[r].s2, c[r].v1, c[r].v2, c[r].vv, c[r].vv2,
                                                 K, fmaf(X.z, kx, gk[r])));
        }
#pragma unroll
        for (int r = 0; r < R; ++r) acc[r] += static_cast<double>(a[r]);
        buf ^= 1;
    }
}

template <int R>
__device__ __forceinline__ void col_pass(const Item *its, const LAUE_GLOBAL float *__restrict__ P1,
                                         const LAUE_GLOBAL float *__restrict__ P2,
                                         const LAUE_GLOBAL Col8 *__restrict__ cols, LAUE_GLOBAL float *__restrict__ G,
                                         const LAUE_GLOBAL float *__restrict__ F0,
                                         const LAUE_GLOBAL float *__restrict__ F1, SinkCtl *__restrict__ ctl,
                                         double2 *__restrict__ part, const SinkParams &p, int n_wg, int n_items,
                                         float *__restrict__ CM) {
    if (ctl->done) return;
    const int k = ctl->iter;
    const LAUE_GLOBAL float *__restrict__ F = (k & 1) ? F1 : F0;
    const double eps = ctl->eps;
    const double kexp = ctl->kexp;
    const float kx = static_cast<float>(kexp);
    const float K = p.twoD2 * kx;
    const double f0 = ctl->f0[k & 1];
    const int r0 = its[0].r0, r1 = its[0].r1;
    int j[R];
    bool act[R];
    Col8 c[R];
    float g[R], gk[R];
    double acc[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        j[r] = its[r].c0 + static_cast<int>(threadIdx.x);
        act[r] = j[r] < its[r].c1;
        c[r] = Col8{0, 0, 0, 0, 1, 1, 1, 0};
        g[r] = 0.0f;
        if (act[r]) {
            c[r] = ld_col(cols + j[r]);
            g[r] = G[j[r]];
        }
        gk[r] = p.part ? static_cast<float>(ctl->H * kexp) : g[r] * kx;
        acc[r] = 0.0;
    }
    // the potentials of state k by parity, each a restrict stream of its own
    if (k & 1)
        col_sums<R>(P1, P2, F1, r0, r1, c, gk, K, kx, acc);
    else
        col_sums<R>(P1, P2, F0, r0, r1, c, gk, K, kx, acc);
    double eb[R], logS[R];
    bool slow[R], any_slow = false;
#pragma unroll
    for (int r = 0; r < R; ++r) {
        eb[r] = (f0 - p.c_unm) * kexp + static_cast<double>(gk[r]);
        acc[r] += exp2(eb[r]);
        slow[r] = act[r] && !(acc[r] > 1e-30 && acc[r] < 1e30);
        any_slow = any_slow || slow[r];
        logS[r] = log(acc[r]);
    }
    if (__any(any_slow)) {
#pragma unroll
        for (int r = 0; r < R; ++r) {
            float mx = static_cast<float>(eb[r]);
            for (int i = r0; i < r1; ++i)
                mx = fmaxf(mx, entry_exponent(P1[i], P2[i], c[r].s1, c[r].s2, c[r].v1, c[r].v2, c[r].vv, c[r].vv2, K,
                                              fmaf(F[i], kx, gk[r])));
            double s2 = exp2(eb[r] - mx);
            for (int i = r0; i < r1; ++i)
                s2 += exp2(static_cast<double>(entry_exponent(P1[i], P2[i], c[r].s1, c[r].s2, c[r].v1, c[r].v2,
                                                              c[r].vv, c[r].vv2, K, fmaf(F[i], kx, gk[r]))) -
                           mx);
            if (slow[r]) logS[r] = log(s2) + static_cast<double>(mx) * 0.6931471805599453;
        }
    }
    const bool unb = p.unb != 0;
    const double tau = unb ? p.lam / (p.lam + eps) : 1.0;
#pragma unroll
    for (int r = 0; r < R; ++r) {
        double cs = 0.0, err = 0.0;
        if (act[r]) {
            const bool empty = r1 <= r0;
            const float gn = p.part ? partial_update(logS[r], eps, empty)
                                    : potential_update(g[r], logS[r], eps, unb, tau, empty);
            G[j[r]] = gn;
            if (p.part) {
                cs = empty ? 0.0 : exp(fmin(logS[r], 0.0));
                err = partial_change(logS[r], g[r], eps, empty, k, CM + j[r]);
            } else {
                cs = exp((f0 + static_cast<double>(gn) - p.c_unm) / eps);
                if (unb) err = mass_change(logS[r], gn, g[r], eps, empty);
            }
        }
        cs = wave_sum(cs);
        err = wave_max(err);
        if (threadIdx.x == 0 && its[r].local >= 0) part[its[r].local] = make_double2(cs, err);
    }
    if (!last_block(ctl, n_wg)) return;
    col_finalize(ctl, part, n_items, p);
}

template <int R>
__global__ __launch_bounds__(64) void k_col(const Item *__restrict__ items, const int2 *__restrict__ groups,
                                            const SampleDesc *__restrict__ descs) {
    Item its[R];
    group_items<R>(items, groups, its);
    const SampleDesc &D = descs[its[0].s];
    col_pass<R>(its, gptr(D.p1), gptr(D.p2), gptr(D.colsE), gptr(D.g), gptr(D.f), gptr(D.f1), D.ctl, D.part,
                D.sp, R == 1 ? D.n_col_items : D.n_col_wg2, D.n_col_items, D.cmass);
}

// ---------------------------------------------------------------- assign

// Hard assignment per detected spot: argmax_j Q_ij over its block and the
// outlier column (lowest index on ties, -1 = outlier), with the sample's final
// potentials and temperature.  Unbalanced OT has no outlier column: the mass
// the plan leaves untransported, max(0, 1 - sum_j Q_ij), takes its place.
__device__ __forceinline__ void assign_pass(const Item &it, const SampleDesc &D,
                                            const LAUE_GLOBAL Col8 *__restrict__ cols,
                                            const LAUE_GLOBAL float *__restrict__ G) {
    const SinkCtl *ctl = D.ctl;
    const SinkParams p = D.sp;
    const double eps = ctl->eps, g0 = ctl->g0[ctl->final_state & 1];
    const int i = it.r0 + static_cast<int>(threadIdx.x);
    const bool act = i < it.r1;
    const double kexp = 1.4426950408889634 / eps;
    const float kx = static_cast<float>(kexp);
    const float K = p.twoD2 * kx;
    const float p1 = act ? D.p1[i] : 0.0f, p2 = act ? D.p2[i] : 0.0f, f = act ? D.f[i] : 0.0f;
    const float fk = f * kx;
    const bool unb = p.unb != 0 || p.part != 0;
    float best = -INFINITY, sum = 0.0f;
    int arg = -1;
    for (int j = it.c0; j < it.c1; ++j) {
        const Col8 c = ld_col(cols + j);
        float e = entry_exponent(p1, p2, c.s1, c.s2, c.v1, c.v2, c.vv, c.vv2, K, fmaf(G[j], kx, fk));
        if (unb) sum += fast_exp2(e);
        if (e > best) {
            best = e;
            arg = j;
        }
    }
    if (!act) return;
    const double eb = (g0 - p.c_out) * kexp + static_cast<double>(fk);
    const float qo = unb ? fmaxf(0.0f, 1.0f - sum) : static_cast<float>(exp2(eb));
    const float qb = arg >= 0 ? fast_exp2(best) : 0.0f;
    const bool m = arg >= 0 && qb >= qo;
    D.jstar[i] = m ? arg : -1;
    D.gstar[i] = m ? D.mgrain[arg] : -1;
    D.qstar[i] = m ? qb : qo;
    D.qout[i] = qo;
}

__global__ __launch_bounds__(64) void k_assign(const Item *__restrict__ items,
                                               const SampleDesc *__restrict__ descs) {
    const Item it = items[blockIdx.x];
    const SampleDesc &D = descs[it.s];
    if (!D.jstar) return;
    assign_pass(it, D, gptr(D.colsE), gptr(D.g));
}

// ---------------------------------------------------------------- M-step

// Per model spot (lane), stream the block's detected spots: the E-step plan
// weight Q_ij (from colsE, at the sample's current temperature) and the
// residual geometry at the current grains (colsC when cur_c, else colsE).
// In the detector frame, with d = v + (p - s), tau = |d|, rhat = d / tau and
// P = I - rhat rhat^T, accumulate
//   S0 = sum Q, e = sum Q (rhat - r), A = sum Q P / tau^2, B = sum Q P / tau
// (rhat - r is formed as ((p - s) - r delta) / tau with
// delta = |d| - |v| = (2 v.(p-s) + |p-s|^2) / (|d| + |v|), free of
// cancellation).  The epilogue turns them into this column's FP64
// contribution to its grain's normal equations:
//   H_ww = D^2 S0 K^T K, H_xx = D^2 Gt^T A Gt, H_xw = D^2 Gt^T B K,
//   g_w = -D^2 K^T e,    g_x = D^2 Gt^T B r,
// with K = 2 (u e^T + (u.e) I) Gt [R w]_x the rotation Jacobian of the ray.
// Statistics per pair of the three M-step passes: 0 Gauss-Newton
// (accumulate_stats), 1 LauePosNewton (accumulate_pos), 2 LaueRotMM
// (accumulate_dir); and each column's FP64 epilogue into colHg.
template <int MODE>
struct MstepMode;
template <>
struct MstepMode<0> {
    static constexpr int N = kStat;
};
template <>
struct MstepMode<1> {
    static constexpr int N = kPosStat;
};
template <>
struct MstepMode<2> {
    static constexpr int N = kDirStat;
};

template <int MODE>
__device__ __forceinline__ void mode_acc(float *a, float Q, float p1, float p2, const Col8 &cC, float vlen, float rn,
                                         float r1, float r2) {
    if constexpr (MODE == 0)
        accumulate_stats(a, Q, p1, p2, cC, vlen, rn, r1, r2);
    else if constexpr (MODE == 1)
        accumulate_pos(a, Q, p1, p2, cC, vlen, rn, r1, r2);
    else
        accumulate_dir(a, Q, p1, p2, cC);
}

template <int MODE>
__device__ __forceinline__ void mode_epilogue(const SampleDesc &D, int j, const double *s64, float rn, float r1,
                                              float r2) {
    double *o = D.colHg + static_cast<int64_t>(j) * kHg;
    if constexpr (MODE == 0)
        column_normal_equations(*D.geom, D.W, D.n_planes, D.grains, D.n_grains, D.mplane[j], D.mgrain[j],
                                D.mblock[j], s64, rn, r1, r2, D.D2, o);
    else if constexpr (MODE == 1)
        column_pos_newton(*D.geom, D.n_grains, D.mgrain[j], D.mblock[j], s64, o);
    else
        column_rot_m0(*D.geom, D.mblock[j], s64, o);
}

// Plan entries at or below this weight (2^-40 of a detected spot's row
// mass) have their M-step statistics skipped; the wave still runs the
// statistics of a row when any of its columns has a larger entry.
constexpr float kMstepMinQ = 0x1p-40f;

template <int MODE>
__device__ __forceinline__ void mstep_pass(const Item &it, const SampleDesc &D,
                                           const LAUE_GLOBAL float *__restrict__ P1,
                                           const LAUE_GLOBAL float *__restrict__ P2,
                                           const LAUE_GLOBAL float *__restrict__ F,
                                           const LAUE_GLOBAL float *__restrict__ G,
                                           const LAUE_GLOBAL Col8 *__restrict__ colsE,
                                           const LAUE_GLOBAL Col8 *__restrict__ colsC, int cur_c) {
    const float kx = static_cast<float>(D.ctl->kexp);
    const float K = D.sp.twoD2 * kx;
    const int j = it.c0 + static_cast<int>(threadIdx.x);
    const bool act = j < it.c1;
    Col8 cE = {0, 0, 0, 0, 1, 1, 1, 0}, cC = {0, 0, 0, 0, 1, 1, 1, 0};
    float g = 0.0f;
    if (act) {
        cE = ld_col(colsE + j);
        if (cur_c) cC = ld_col(colsC + j); else cC = cE;
        g = G[j];
    }
    const float gk = g * kx;
    const float ivl = __builtin_amdgcn_rsqf(cC.vv);
    const float vlen = cC.vv * ivl;
    const float rn = cC.vn * ivl, r1 = cC.v1 * ivl, r2 = cC.v2 * ivl;
    constexpr int NS = MstepMode<MODE>::N;
    double s64[NS];
    for (int k = 0; k < NS; ++k) s64[k] = 0.0;
    // 64 rows at a time through LDS (p1, p2, f of row i0 + lane), read back
    // by broadcast LDS loads, the next chunk's loads in flight meanwhile
    __shared__ float4 lr[2][64];
    const int lane = static_cast<int>(threadIdx.x);
    float4 nx = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    if (it.r0 + lane < it.r1) nx = make_float4(P1[it.r0 + lane], P2[it.r0 + lane], F[it.r0 + lane], 0.0f);
    int buf = 0;
    for (int i0 = it.r0; i0 < it.r1; i0 += 64) {
        const int ni = min(64, it.r1 - i0);
        lr[buf][lane] = nx;
        __syncthreads();
        const int in = i0 + 64 + lane;
        if (in < it.r1) nx = make_float4(P1[in], P2[in], F[in], 0.0f);
        float a[NS];
        for (int k = 0; k < NS; ++k) a[k] = 0.0f;
#pragma unroll 4
        for (int t = 0; t < ni; ++t) {
            const float4 X = lr[buf][t];
            const float Q = fast_exp2(entry_exponent(X.x, X.y, cE.s1, cE.s2, cE.v1, cE.v2, cE.vv,
                                                     cE.vv2, K, fmaf(X.z, kx, gk)));
            if (Q > kMstepMinQ) mode_acc<MODE>(a, Q, X.x, X.y, cC, vlen, rn, r1, r2);
        }
        for (int k = 0; k < NS; ++k) s64[k] += static_cast<double>(a[k]);
        buf ^= 1;
    }
    if (!act) return;
    mode_epilogue<MODE>(D, j, s64, rn, r1, r2);
}

template <int MODE>
__global__ __launch_bounds__(64) void k_mstep_acc(const Item *__restrict__ items,
                                                  const SampleDesc *__restrict__ descs, int cur_c) {
    const Item it = items[blockIdx.x];
    const SampleDesc &D = descs[it.s];
    mstep_pass<MODE>(it, D, gptr(D.p1), gptr(D.p2), gptr(D.f), gptr(D.g), gptr(D.colsE), gptr(D.colsC), cur_c);
}

// One wave per grain of any sample (gbase: grain offsets of the samples):
// sum its columns' contributions (per block, the grain's columns are one
// contiguous run found by binary search), then lane 0 solves
// (H + mu I) step = -g by Cholesky in FP64 and applies the step.
__global__ __launch_bounds__(64) void k_mstep_solve(const SampleDesc *__restrict__ descs, int n_samples,
                                                    const int64_t *__restrict__ gbase) {
    const int s = sample_of(gbase, n_samples, blockIdx.x);
    const SampleDesc &D = descs[s];
    const int n = static_cast<int>(blockIdx.x - gbase[s]);
    const int *__restrict__ mgrain = D.mgrain;
    double acc[kHg];
    for (int k = 0; k < kHg; ++k) acc[k] = 0.0;
    for (int b = threadIdx.x; b < D.nb; b += 64) {
        int64_t lo = D.mboff[b], hi = D.mboff[b + 1];
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
            for (int k = 0; k < kHg; ++k) acc[k] += D.colHg[j * kHg + k];
    }
    for (int k = 0; k < kHg; ++k) acc[k] = wave_sum(acc[k]);
    if (threadIdx.x != 0) return;
    gn_solve_apply(acc, D.mu_rel, D.q + 4 * n, D.x + 3 * n, D.grains + n,
                   D.step_norm ? D.step_norm + n : nullptr);
}

// the contiguous run [a, z) of grain n's columns in block b (columns of a
// block ascend by grain)
__device__ __forceinline__ void grain_run(const SampleDesc &D, int b, int n, int64_t &a, int64_t &z) {
    const int *__restrict__ mgrain = D.mgrain;
    const int64_t lo = D.mboff[b], hi = D.mboff[b + 1];
    int64_t e = hi;
    a = lo;
    while (a < e) {
        const int64_t mid = (a + e) >> 1;
        if (mgrain[mid] < n) a = mid + 1; else e = mid;
    }
    z = a;
    e = hi;
    while (z < e) {
        const int64_t mid = (z + e) >> 1;
        if (mgrain[mid] <= n) z = mid + 1; else e = mid;
    }
}

// LauePosNewton step it of one grain (one wave per grain of any sample): sum
// its columns' (H_x, g_x) as k_mstep_solve does, then lane 0 applies
// x <- x - H_x^-1 g_x (FP64, by the adjugate; a singular H_x is skipped).  A
// grain whose step fell below tol_x takes no further step in this sweep
// (it == 0 starts the sweep).
__global__ __launch_bounds__(64) void k_pos_solve(const SampleDesc *__restrict__ descs, int n_samples,
                                                  const int64_t *__restrict__ gbase, int it) {
    const int s = sample_of(gbase, n_samples, blockIdx.x);
    const SampleDesc &D = descs[s];
    const int n = static_cast<int>(blockIdx.x - gbase[s]);
    double acc[kPosStat];
    for (int k = 0; k < kPosStat; ++k) acc[k] = 0.0;
    for (int b = threadIdx.x; b < D.nb; b += 64) {
        int64_t a, z;
        grain_run(D, b, n, a, z);
        for (int64_t j = a; j < z; ++j)
            for (int k = 0; k < kPosStat; ++k) acc[k] += D.colHg[j * kHg + k];
    }
    for (int k = 0; k < kPosStat; ++k) acc[k] = wave_sum(acc[k]);
    if (threadIdx.x != 0) return;
    int *flag = D.gflag + n;
    if (it == 0) *flag = 0;
    else if (*flag) return;
    const double h00 = acc[0], h01 = acc[1], h02 = acc[2], h11 = acc[3], h12 = acc[4], h22 = acc[5];
    const double c00 = h11 * h22 - h12 * h12, c01 = h02 * h12 - h01 * h22, c02 = h01 * h12 - h02 * h11;
    const double c11 = h00 * h22 - h02 * h02, c12 = h01 * h02 - h00 * h12, c22 = h00 * h11 - h01 * h01;
    const double det = h00 * c00 + h01 * c01 + h02 * c02;
    const double scale = fabs(h00) + fabs(h11) + fabs(h22);
    if (!(fabs(det) > 1e-14 * scale * scale * scale) || !isfinite(det)) return;
    const double g0 = acc[6], g1 = acc[7], g2 = acc[8];
    const double dx[3] = {(c00 * g0 + c01 * g1 + c02 * g2) / det, (c01 * g0 + c11 * g1 + c12 * g2) / det,
                          (c02 * g0 + c12 * g1 + c22 * g2) / det};
    double *x = D.x + 3 * n;
    for (int k = 0; k < 3; ++k) x[k] -= dx[k];
    D.grains[n] = grain_f32(D.q + 4 * n, x);
    const double nd = sqrt(dx[0] * dx[0] + dx[1] * dx[1] + dx[2] * dx[2]);
    if (D.step_norm) D.step_norm[n] = nd;
    if (nd < D.tol_x) *flag = 1;
}

// LaueRotMM of one grain (one wave per grain of any sample).  M0 per plane
// (Eq. M0) is summed in LDS from the grain's columns, block by block in
// order (lanes 0..5 each own one of the six entries, so the sum has a fixed
// order); each M0 is shifted by the magnitude of its smallest eigenvalue when
// that is negative (Eq. Mm); then R <- Wahba(M_m R w_m, w_m, 1) (Eq.
// majmin_step) until ||R' - R||_F < tol_r or k_mm steps, with B = sum_m
// (M_m R w_m) w_m^T summed over the lanes' planes and one fixed wave
// reduction, so that every lane solves the same Wahba problem.
__global__ __launch_bounds__(64) void k_rot_mm(const SampleDesc *__restrict__ descs, int n_samples,
                                               const int64_t *__restrict__ gbase) {
    __shared__ double Msh[kMaxPlanesMM * 6];
    const int s = sample_of(gbase, n_samples, blockIdx.x);
    const SampleDesc &D = descs[s];
    const int n = static_cast<int>(blockIdx.x - gbase[s]);
    const int np = min(D.n_planes, kMaxPlanesMM);
    const int lane = threadIdx.x;
    for (int k = lane; k < np * 6; k += 64) Msh[k] = 0.0;
    __syncthreads();
    if (lane < 6) {
        for (int b = 0; b < D.nb; ++b) {
            int64_t a, z;
            grain_run(D, b, n, a, z);
            for (int64_t j = a; j < z; ++j) {
                const int m = D.mplane[j];
                if (m >= 0 && m < np) Msh[6 * m + lane] += D.colHg[j * kHg + lane];
            }
        }
    }
    __syncthreads();
    for (int m = lane; m < np; m += 64) {
        double *M = Msh + 6 * m;
        const double lmin = sym3_min_eig(M);
        if (lmin < 0.0) {
            M[0] -= lmin;
            M[3] -= lmin;
            M[5] -= lmin;
        }
    }
    __syncthreads();
    double q[4] = {D.q[4 * n], D.q[4 * n + 1], D.q[4 * n + 2], D.q[4 * n + 3]};
    const double qn0 = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
    for (int k = 0; k < 4; ++k) q[k] /= qn0;
    double R[9];
    quat_R(q, R);
    bool moved = false;
    for (int it = 0; it < D.k_mm; ++it) {
        double Bl[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
        for (int m = lane; m < np; m += 64) {
            const double *M = Msh + 6 * m;
            if (M[0] == 0.0 && M[1] == 0.0 && M[2] == 0.0 && M[3] == 0.0 && M[4] == 0.0 && M[5] == 0.0) continue;
            const double w[3] = {D.W[3 * m], D.W[3 * m + 1], D.W[3 * m + 2]};
            const double v[3] = {R[0] * w[0] + R[1] * w[1] + R[2] * w[2], R[3] * w[0] + R[4] * w[1] + R[5] * w[2],
                                 R[6] * w[0] + R[7] * w[1] + R[8] * w[2]};
            const double av[3] = {M[0] * v[0] + M[1] * v[1] + M[2] * v[2], M[1] * v[0] + M[3] * v[1] + M[4] * v[2],
                                  M[2] * v[0] + M[4] * v[1] + M[5] * v[2]};
            for (int a_ = 0; a_ < 3; ++a_)
                for (int b_ = 0; b_ < 3; ++b_) Bl[3 * a_ + b_] += av[a_] * w[b_];
        }
        double B[3][3], bn = 0.0;
        for (int k = 0; k < 9; ++k) {
            B[k / 3][k % 3] = wave_sum(Bl[k]);
            bn += B[k / 3][k % 3] * B[k / 3][k % 3];
        }
        if (!(bn > 0.0) || !isfinite(bn)) break;
        double qn[4], Rn[9];
        wahba_quat_B(B, qn);
        quat_R(qn, Rn);
        double z = 0.0;
        for (int k = 0; k < 9; ++k) z += (Rn[k] - R[k]) * (Rn[k] - R[k]);
        for (int k = 0; k < 9; ++k) R[k] = Rn[k];
        for (int k = 0; k < 4; ++k) q[k] = qn[k];
        moved = true;
        if (sqrt(z) < D.tol_r) break;
    }
    if (lane != 0 || !moved) return;
    for (int k = 0; k < 4; ++k) D.q[4 * n + k] = q[k];
    D.grains[n] = grain_f32(q, D.x + 3 * n);
}

// ---------------------------------------------------------------- sparse assignment

// Each detected spot keeps its rho nearest model spots of its block by the
// chord cost (ties to the lower model-spot index); the plan is null outside
// these sets (Sec. 5.2).  The sets are chosen afresh before every Sinkhorn
// from the packed columns of that E-step (colsE).  Row side: nbr / ncp
// [rho x n_obs], neighbour-major so that a wave's rows read adjacent words
// (model-spot index or -1, c' = c / (2 D^2)), ordered by (c', index).  Column side: CSR by model spot (col_off, col_row, col_cp),
// rows ascending.

// insert (x, xj) into the sorted register list (d, id) of length R; the last
// entry falls off.  Candidates arrive in ascending index, so strict < keeps
// the lower index on equal costs.
template <int R>
__device__ __forceinline__ void knn_insert(float *d, int *id, float x, int xj) {
#pragma unroll
    for (int k = 0; k < R; ++k) {
        const bool sw = x < d[k];
        const float td = sw ? d[k] : x;
        const int tj = sw ? id[k] : xj;
        d[k] = sw ? x : d[k];
        id[k] = sw ? xj : id[k];
        x = td;
        xj = tj;
    }
}

// Filter pass (lane = detected spot of a 64-row item): every column of the
// block with c' below the block's threshold is appended to the row's
// candidate list (at most M kept; the count is exact).
__device__ __forceinline__ void knn_filter_body(const Item &it, const LAUE_GLOBAL float *__restrict__ P1,
                                                const LAUE_GLOBAL float *__restrict__ P2,
                                                const LAUE_GLOBAL Col8 *__restrict__ cols, int *__restrict__ cj,
                                                float *__restrict__ cc, int *__restrict__ cnt_out, int M,
                                                float thr, int64_t n_obs) {
    const int i = it.r0 + static_cast<int>(threadIdx.x);
    const bool act = i < it.r1;
    const float p1 = act ? P1[i] : 0.0f, p2 = act ? P2[i] : 0.0f;
    int cnt = 0;
    const int64_t base = act ? i : 0;   // candidate-major: candidate t of row i at t n_obs + i
    for (int j = it.c0; j < it.c1; ++j) {
        const Col8 c = ld_col(cols + j);
        const float cp = chord_cp(p1, p2, c.s1, c.s2, c.v1, c.v2, c.vv, c.vv2);
        if (act && cp < thr) {
            if (cnt < M) {
                cj[cnt * n_obs + base] = j;
                cc[cnt * n_obs + base] = cp;
            }
            ++cnt;
        }
    }
    if (act) cnt_out[i] = cnt;
}

// Density grid of the model spots: kGrid x kGrid cells per block over the
// detector square (detector-local coordinates).
constexpr int kGrid = 16;

__device__ __forceinline__ int grid_cell(float u, float half) {
    const float t = (u + half) * (static_cast<float>(kGrid) / (2.0f * half));
    return min(max(static_cast<int>(floorf(t)), 0), kGrid - 1);
}

__global__ void k_knn_hist(const SampleDesc *__restrict__ descs, int s) {
    const SampleDesc &D = descs[s];
    const int64_t j = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (j >= D.n_model) return;
    const int b = D.mblock[j];
    if (b < 0 || b >= D.nb) return;
    const float half = D.geom->det[b % D.geom->n_det].half;
    const Col8 c = D.colsE[j];
    if (!(c.s1 == c.s1) || !(c.s2 == c.s2)) return;
    atomicAdd(D.knn_hist + b * kGrid * kGrid + grid_cell(c.s2, half) * kGrid + grid_cell(c.s1, half), 1);
}

// Per-row filter threshold: 3 rho model spots expected within it at the
// local density of the 3x3 cells around the row (pi r^2 lambda = 3 rho,
// c' ~ r^2 / (2 D^2) near normal incidence); the block's mean density where
// those cells are empty.
__device__ __forceinline__ float knn_threshold(const SampleDesc &D, int b, float p1, float p2, int Jb) {
    const float half = D.geom->det[b % D.geom->n_det].half;
    const int cx = grid_cell(p1, half), cy = grid_cell(p2, half);
    int c9 = 0, n9 = 0;
    for (int dy = -1; dy <= 1; ++dy)
        for (int dx = -1; dx <= 1; ++dx) {
            const int x = cx + dx, y = cy + dy;
            if (x < 0 || x >= kGrid || y < 0 || y >= kGrid) continue;
            c9 += D.knn_hist[b * kGrid * kGrid + y * kGrid + x];
            ++n9;
        }
    const float h = 2.0f * half / static_cast<float>(kGrid);
    const float lambda = c9 > 0 ? static_cast<float>(c9) / (static_cast<float>(n9) * h * h)
                                : static_cast<float>(Jb) / (4.0f * half * half);
    return static_cast<float>(3.0 * D.rho / (M_PI * lambda * 2.0 * D.D2));
}

__global__ __launch_bounds__(64) void k_knn_filter(const Item *__restrict__ items,
                                                   const SampleDesc *__restrict__ descs) {
    const Item it = items[blockIdx.x];
    const SampleDesc &D = descs[it.s];
    const int Jb = it.c1 - it.c0;
    if (Jb <= D.rho) return;      // every column is a neighbour: the exact pass takes the row
    // the item's block: the last b with oboff[b] <= r0
    int lo = 0, hi = D.nb;
    while (hi - lo > 1) {
        const int mid = (lo + hi) / 2;
        if (D.oboff[mid] <= it.r0) lo = mid; else hi = mid;
    }
    const int i = it.r0 + static_cast<int>(threadIdx.x);
    const float thr = i < it.r1 ? knn_threshold(D, lo, D.p1[i], D.p2[i], Jb) : 0.0f;
    knn_filter_body(it, gptr(D.p1), gptr(D.p2), gptr(D.colsE), D.cand_j, D.cand_c, D.cand_n, D.cand_cap, thr,
                    D.n_obs);
}

// Selection (lane = detected spot): the rho smallest of the row's candidates
// when the filter kept at least rho and at most M of them (then they hold the
// true rho nearest: every column not kept has c' >= the threshold > the
// rho-th kept); otherwise the row goes to the exact pass.
template <int R>
__global__ __launch_bounds__(64) void k_knn_select(const Item *__restrict__ items,
                                                   const SampleDesc *__restrict__ descs) {
    const Item it = items[blockIdx.x];
    const SampleDesc &D = descs[it.s];
    const int i = it.r0 + static_cast<int>(threadIdx.x);
    if (i >= it.r1) return;
    const int Jb = it.c1 - it.c0;
    const int n = Jb <= R ? -1 : D.cand_n[i];
    if (n < R || n > D.cand_cap) {
        D.knn_list[atomicAdd(D.knn_nlist, 1)] = i;
        return;
    }
    float d[R];
    int id[R];
#pragma unroll
    for (int k = 0; k < R; ++k) {
        d[k] = INFINITY;
        id[k] = -1;
    }
    for (int t = 0; t < n; ++t) knn_insert<R>(d, id, D.cand_c[t * D.n_obs + i], D.cand_j[t * D.n_obs + i]);
#pragma unroll
    for (int k = 0; k < R; ++k) {
        D.nbr[k * D.n_obs + i] = id[k];
        D.ncp[k * D.n_obs + i] = d[k];
    }
}

// Exact pass over the listed rows (lane = one listed row; the rows of a wave
// may lie in different blocks): all columns of the row's block.
template <int R>
__global__ __launch_bounds__(64) void k_knn_exact(const SampleDesc *__restrict__ descs, int s, int n_list) {
    const SampleDesc &D = descs[s];
    const int t = blockIdx.x * 64 + static_cast<int>(threadIdx.x);
    if (t >= n_list) return;
    const int i = D.knn_list[t];
    // block of row i: the last b with oboff[b] <= i
    int lo = 0, hi = D.nb;
    while (hi - lo > 1) {
        const int mid = (lo + hi) / 2;
        if (D.oboff[mid] <= i) lo = mid; else hi = mid;
    }
    const int c0 = static_cast<int>(D.mboff[lo]), c1 = static_cast<int>(D.mboff[lo + 1]);
    const float p1 = D.p1[i], p2 = D.p2[i];
    float d[R];
    int id[R];
#pragma unroll
    for (int k = 0; k < R; ++k) {
        d[k] = INFINITY;
        id[k] = -1;
    }
    for (int j = c0; j < c1; ++j) {
        const Col8 c = D.colsE[j];
        knn_insert<R>(d, id, chord_cp(p1, p2, c.s1, c.s2, c.v1, c.v2, c.vv, c.vv2), j);
    }
#pragma unroll
    for (int k = 0; k < R; ++k) {
        D.nbr[k * D.n_obs + i] = id[k];
        D.ncp[k * D.n_obs + i] = d[k];
    }
}

// Column lists: the entries are ordered by model spot with a stable radix
// sort (every list then has a fixed order and the sums over it are
// reproducible); the offsets are found by binary search in the sorted keys.
// radix-sort input: key = model spot (n_model for an empty slot), value = entry
__global__ void k_knn_keys(const SampleDesc *__restrict__ descs, int s) {
    const SampleDesc &D = descs[s];
    const int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (e >= D.n_obs * D.rho) return;
    const int j = D.nbr[e];
    D.sort_key[e] = j >= 0 ? j : static_cast<int>(D.n_model);
    D.sort_val[e] = static_cast<int>(e);
}

// column offsets from the sorted keys: col_off[j] = first sorted entry with
// key >= j (keys of empty slots are n_model and sort last)
__global__ void k_knn_offsets(const SampleDesc *__restrict__ descs, int s, const int *__restrict__ skey) {
    const SampleDesc &D = descs[s];
    const int64_t j = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (j > D.n_model) return;
    int64_t lo = 0, hi = D.n_obs * D.rho;
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (skey[mid] < j) lo = mid + 1; else hi = mid;
    }
    D.col_off[j] = lo;
}

// column lists from the entries sorted by model spot (stable: within a
// column, entries keep their neighbour-major order)
__global__ void k_knn_gather(const SampleDesc *__restrict__ descs, int s) {
    const SampleDesc &D = descs[s];
    const int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (t >= D.col_off[D.n_model]) return;
    const int e = D.sorted_val[t];
    D.col_row[t] = static_cast<int>(e % D.n_obs);
    D.col_cp[t] = D.ncp[e];
}

// neighbour-major sets to row-major output ([n_obs x rho]), costs in mm^2
__global__ void k_knn_out(const int *__restrict__ nbr, const float *__restrict__ ncp, int64_t n_obs, int rho,
                          float twoD2, int *__restrict__ onbr, float *__restrict__ ocost) {
    const int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (e >= n_obs * rho) return;
    const int64_t i = e / rho, q = e % rho;
    onbr[e] = nbr[q * n_obs + i];
    ocost[e] = ncp[q * n_obs + i] * twoD2;
}

// x[k] = v (partial OT: the Gibbs-kernel start) or x[k] += v (folding the
// mass potential into the row potentials), k < n
__global__ void k_fill_f(float *__restrict__ x, int64_t n, double v, int add) {
    const int64_t k = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (k < n) x[k] = add ? static_cast<float>(static_cast<double>(x[k]) + v) : static_cast<float>(v);
}

__global__ void k_zero_i(int *__restrict__ p, int64_t n) {
    const int64_t k = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (k < n) p[k] = 0;
}

// Sparse row half (lane = detected spot): S_i over the row's neighbours, then
// the dense pass's epilogue and finalisation.
__global__ __launch_bounds__(64) void k_row_sparse(const Item *__restrict__ items,
                                                   const SampleDesc *__restrict__ descs) {
    const Item it = items[blockIdx.x];
    const SampleDesc &D = descs[it.s];
    SinkCtl *ctl = D.ctl;
    if (ctl->done) return;
    const SinkParams &p = D.sp;
    const int k = ctl->iter + 1;
    const float *Fin = ((k - 1) & 1) ? D.f1 : D.f;
    float *Fout = (k & 1) ? D.f1 : D.f;
    const double eps = ctl->eps;
    const double kexp = ctl->kexp;
    const float kx = static_cast<float>(kexp);
    const float K = p.twoD2 * kx;
    const double g0 = ctl->g0[(k - 1) & 1];
    const int R = D.rho;
    const int i = it.r0 + static_cast<int>(threadIdx.x);
    const bool act = i < it.r1;
    const float f = act ? Fin[i] : 0.0f;
    const float fk = p.part ? static_cast<float>(ctl->H * kexp) : f * kx;
    const int64_t base = act ? i : 0, st = D.n_obs;   // neighbour-major: entry q of row i at q n_obs + i
    float a = 0.0f;
    for (int q = 0; q < R; ++q) {
        const int j = act ? D.nbr[q * st + base] : -1;
        if (j >= 0) a += fast_exp2(fmaf(-K, D.ncp[q * st + base], fmaf(D.g[j], kx, fk)));
    }
    double acc = static_cast<double>(a);
    const double eb = (g0 - p.c_out) * kexp + static_cast<double>(fk);
    acc += exp2(eb);
    const bool slow = act && !(acc > 1e-30 && acc < 1e30);
    double logS = log(acc);
    if (__any(slow) && slow) {
        float mx = static_cast<float>(eb);
        for (int q = 0; q < R; ++q) {
            const int j = D.nbr[q * st + base];
            if (j >= 0) mx = fmaxf(mx, fmaf(-K, D.ncp[q * st + base], fmaf(D.g[j], kx, fk)));
        }
        double s2 = exp2(eb - mx);
        for (int q = 0; q < R; ++q) {
            const int j = D.nbr[q * st + base];
            if (j >= 0)
                s2 += exp2(static_cast<double>(fmaf(-K, D.ncp[q * st + base], fmaf(D.g[j], kx, fk))) - mx);
        }
        logS = log(s2) + static_cast<double>(mx) * 0.6931471805599453;
    }
    const bool unb = p.unb != 0;
    const bool empty = !act || D.nbr[base] < 0;
    const float fnf = p.part ? partial_update(logS, eps, empty)
                             : potential_update(f, logS, eps, unb, unb ? p.kappa / (p.kappa + eps) : 1.0, empty);
    double err = !act     ? 0.0
                 : p.part ? partial_change(logS, f, eps, empty, k, D.rmass + i)
                 : unb    ? mass_change(logS, fnf, f, eps, empty)
                          : fabs(acc - 1.0);
    double rs = 0.0;
    if (act) {
        Fout[i] = fnf;
        rs = exp((static_cast<double>(fnf) + g0 - p.c_out) / eps);
    }
    rs = wave_sum(rs);
    err = wave_max(err);
    if (threadIdx.x == 0) D.part[it.local] = make_double2(rs, err);
    if (!last_block(ctl, D.n_row_items)) return;
    row_finalize(ctl, D.part, p, D.n_row_items, k, eps);
}

// Sparse column half (lane = model spot): over the rows that keep it.
__global__ __launch_bounds__(64) void k_col_sparse(const Item *__restrict__ items,
                                                   const SampleDesc *__restrict__ descs) {
    const Item it = items[blockIdx.x];
    const SampleDesc &D = descs[it.s];
    SinkCtl *ctl = D.ctl;
    if (ctl->done) return;
    const SinkParams &p = D.sp;
    const int k = ctl->iter;
    const float *F = (k & 1) ? D.f1 : D.f;
    const double eps = ctl->eps;
    const double kexp = ctl->kexp;
    const float kx = static_cast<float>(kexp);
    const float K = p.twoD2 * kx;
    const double f0 = ctl->f0[k & 1];
    const int j = it.c0 + static_cast<int>(threadIdx.x);
    const bool act = j < it.c1;
    const float g = act ? D.g[j] : 0.0f;
    const float gk = p.part ? static_cast<float>(ctl->H * kexp) : g * kx;
    const int64_t a0 = act ? D.col_off[j] : 0, a1 = act ? D.col_off[j + 1] : 0;
    float a = 0.0f;
    for (int64_t e = a0; e < a1; ++e) a += fast_exp2(fmaf(-K, D.col_cp[e], fmaf(F[D.col_row[e]], kx, gk)));
    double acc = static_cast<double>(a);
    const double eb = (f0 - p.c_unm) * kexp + static_cast<double>(gk);
    acc += exp2(eb);
    const bool slow = act && !(acc > 1e-30 && acc < 1e30);
    double logS = log(acc);
    if (__any(slow) && slow) {
        float mx = static_cast<float>(eb);
        for (int64_t e = a0; e < a1; ++e) mx = fmaxf(mx, fmaf(-K, D.col_cp[e], fmaf(F[D.col_row[e]], kx, gk)));
        double s2 = exp2(eb - mx);
        for (int64_t e = a0; e < a1; ++e)
            s2 += exp2(static_cast<double>(fmaf(-K, D.col_cp[e], fmaf(F[D.col_row[e]], kx, gk))) - mx);
        logS = log(s2) + static_cast<double>(mx) * 0.6931471805599453;
    }
    const bool unb = p.unb != 0;
    double cs = 0.0, err = 0.0;
    if (act) {
        const bool empty = a1 <= a0;
        const float gn = p.part ? partial_update(logS, eps, empty)
                                : potential_update(g, logS, eps, unb, unb ? p.lam / (p.lam + eps) : 1.0, empty);
        D.g[j] = gn;
        if (p.part) {
            cs = empty ? 0.0 : exp(fmin(logS, 0.0));
            err = partial_change(logS, g, eps, empty, k, D.cmass + j);
        } else {
            cs = exp((f0 + static_cast<double>(gn) - p.c_unm) / eps);
            if (unb) err = mass_change(logS, gn, g, eps, empty);
        }
    }
    cs = wave_sum(cs);
    err = wave_max(err);
    if (threadIdx.x == 0) D.part[it.local] = make_double2(cs, err);
    if (!last_block(ctl, D.n_col_items)) return;
    col_finalize(ctl, D.part, D.n_col_items, p);
}

// Sparse M-step statistics (lane = model spot): over the rows that keep it,
// Q from the stored E-step cost and the potentials, the residual geometry at
// the current grains; same epilogue as the dense pass.
template <int MODE>
__global__ __launch_bounds__(64) void k_mstep_acc_sparse(const Item *__restrict__ items,
                                                         const SampleDesc *__restrict__ descs, int cur_c) {
    const Item it = items[blockIdx.x];
    const SampleDesc &D = descs[it.s];
    const float kx = static_cast<float>(D.ctl->kexp);
    const float K = D.sp.twoD2 * kx;
    const int j = it.c0 + static_cast<int>(threadIdx.x);
    const bool act = j < it.c1;
    Col8 cC = {0, 0, 0, 0, 1, 1, 1, 0};
    float g = 0.0f;
    if (act) {
        cC = cur_c ? D.colsC[j] : D.colsE[j];
        g = D.g[j];
    }
    const float gk = g * kx;
    const float ivl = __builtin_amdgcn_rsqf(cC.vv);
    const float vlen = cC.vv * ivl;
    const float rn = cC.vn * ivl, r1 = cC.v1 * ivl, r2 = cC.v2 * ivl;
    const int64_t a0 = act ? D.col_off[j] : 0, a1 = act ? D.col_off[j + 1] : 0;
    constexpr int NS = MstepMode<MODE>::N;
    float a[NS];
    for (int q = 0; q < NS; ++q) a[q] = 0.0f;
    for (int64_t e = a0; e < a1; ++e) {
        const int i = D.col_row[e];
        const float Q = fast_exp2(fmaf(-K, D.col_cp[e], fmaf(D.f[i], kx, gk)));
        if (Q > 0.0f) mode_acc<MODE>(a, Q, D.p1[i], D.p2[i], cC, vlen, rn, r1, r2);
    }
    if (!act) return;
    double s64[NS];
    for (int q = 0; q < NS; ++q) s64[q] = static_cast<double>(a[q]);
    mode_epilogue<MODE>(D, j, s64, rn, r1, r2);
}

// Sparse hard assignment: argmax over the row's neighbours (lowest index on
// ties) and the outlier column (unbalanced OT: the untransported mass).
__global__ __launch_bounds__(64) void k_assign_sparse(const Item *__restrict__ items,
                                                      const SampleDesc *__restrict__ descs) {
    const Item it = items[blockIdx.x];
    const SampleDesc &D = descs[it.s];
    if (!D.jstar) return;
    const SinkCtl *ctl = D.ctl;
    const SinkParams p = D.sp;
    const double eps = ctl->eps, g0 = ctl->g0[ctl->final_state & 1];
    const int i = it.r0 + static_cast<int>(threadIdx.x);
    if (i >= it.r1) return;
    const double kexp = 1.4426950408889634 / eps;
    const float kx = static_cast<float>(kexp);
    const float K = p.twoD2 * kx;
    const float fk = D.f[i] * kx;
    const bool unb = p.unb != 0 || p.part != 0;
    float best = -INFINITY, sum = 0.0f;
    int arg = -1;
    for (int q = 0; q < D.rho; ++q) {
        const int j = D.nbr[q * D.n_obs + i];
        if (j < 0) continue;
        const float e = fmaf(-K, D.ncp[q * D.n_obs + i], fmaf(D.g[j], kx, fk));
        if (unb) sum += fast_exp2(e);
        if (e > best || (e == best && j < arg)) {
            best = e;
            arg = j;
        }
    }
    const double eb = (g0 - p.c_out) * kexp + static_cast<double>(fk);
    const float qo = unb ? fmaxf(0.0f, 1.0f - sum) : static_cast<float>(exp2(eb));
    const float qb = arg >= 0 ? fast_exp2(best) : 0.0f;
    const bool m = arg >= 0 && qb >= qo;
    D.jstar[i] = m ? arg : -1;
    D.gstar[i] = m ? D.mgrain[arg] : -1;
    D.qstar[i] = m ? qb : qo;
    D.qout[i] = qo;
}

// ---------------------------------------------------------------- forward model

// FP32 grains of all samples from their FP64 quaternions and positions.
__global__ void k_grain_prep_b(const SampleDesc *__restrict__ descs, int n_samples,
                               const int64_t *__restrict__ gbase) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= gbase[n_samples]) return;
    const int s = sample_of(gbase, n_samples, i);
    const SampleDesc &D = descs[s];
    const int64_t n = i - gbase[s];
    D.grains[n] = grain_f32(D.q + 4 * n, D.x + 3 * n);
}

// Forward model on the frozen model-spot lists of all samples (mbase: model
// offsets of the samples): the model arrays (when present) and the packed
// columns colsE (to_c = 0) or colsC (to_c = 1).
__global__ void k_eval_b(const SampleDesc *__restrict__ descs, int n_samples, const int64_t *__restrict__ mbase,
                         int to_c, int with_outputs) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= mbase[n_samples]) return;
    const int s = sample_of(mbase, n_samples, i);
    const SampleDesc &D = descs[s];
    const int64_t j = i - mbase[s];
    const GeomF &G = *D.geom;
    Col8 *cols = to_c ? D.colsC : D.colsE;
    const int m = D.mplane[j], g = D.mgrain[j], b = D.mblock[j];
    if (m < 0 || m >= D.n_planes || g < 0 || g >= D.n_grains || b < 0 || b >= G.n_rot * G.n_det) {
        // invalid ids: no geometry (NaN) rather than an out-of-bounds read
        const float nan = __builtin_nanf("");
        if (with_outputs && D.s1) { D.s1[j] = nan; D.s2[j] = nan; D.vn[j] = nan; D.v1[j] = nan; D.v2[j] = nan; }
        if (with_outputs && D.lam) D.lam[j] = nan;
        cols[j] = Col8{nan, nan, nan, nan, nan, nan, nan, 0.0f};
        return;
    }
    const int t = b / G.n_det, d = b - t * G.n_det;
    const GrainF &gr = D.grains[g];
    const SpotGeo o = spot_geometry(G, G.det[d], gr.R, gr.x, G.cs[t][0], G.cs[t][1], D.W[3 * m],
                                    D.W[3 * m + 1], D.W[3 * m + 2], D.Dsp[m]);
    if (with_outputs && D.s1) {
        D.s1[j] = o.s1;
        D.s2[j] = o.s2;
        D.vn[j] = o.vn;
        D.v1[j] = o.v1;
        D.v2[j] = o.v2;
    }
    if (with_outputs && D.lam) D.lam[j] = o.lam;
    Col8 c;
    c.s1 = o.s1;
    c.s2 = o.s2;
    c.v1 = o.v1;
    c.v2 = o.v2;
    c.vv = fmaf(o.v2, o.v2, fmaf(o.v1, o.v1, o.vn * o.vn));
    c.vv2 = c.vv * c.vv;
    c.vn = o.vn;
    c.pad = 0.0f;
    cols[j] = c;
}

// ---------------------------------------------------------------- host side

struct SamplePlan {
    std::vector<Item> rows, cols;
    int64_t entries = 0;   // sum_b I_b J_b
};

static SamplePlan make_plan(const int64_t *ob, const int64_t *mb, int nb, int s) {
    SamplePlan p;
    for (int b = 0; b < nb; ++b) {
        int r0 = static_cast<int>(ob[b]), r1 = static_cast<int>(ob[b + 1]);
        int c0 = static_cast<int>(mb[b]), c1 = static_cast<int>(mb[b + 1]);
        p.entries += static_cast<int64_t>(r1 - r0) * (c1 - c0);
        for (int r = r0; r < r1; r += 64) p.rows.push_back({r, std::min(r + 64, r1), c0, c1, s, 0, {0, 0}});
        for (int c = c0; c < c1; c += 64) p.cols.push_back({r0, r1, c, std::min(c + 64, c1), s, 0, {0, 0}});
    }
    // a pass always has at least one (possibly empty) workgroup per sample:
    // the last one finalises the sample's bins
    if (p.rows.empty()) p.rows.push_back({0, 0, 0, 0, s, 0, {0, 0}});
    if (p.cols.empty()) p.cols.push_back({0, 0, 0, 0, s, 0, {0, 0}});
    // heaviest items first so the tail of the grid is short
    std::stable_sort(p.rows.begin(), p.rows.end(),
                     [](const Item &a, const Item &b) { return (a.c1 - a.c0) > (b.c1 - b.c0); });
    std::stable_sort(p.cols.begin(), p.cols.end(),
                     [](const Item &a, const Item &b) { return (a.r1 - a.r0) > (b.r1 - b.r0); });
    for (size_t k = 0; k < p.rows.size(); ++k) p.rows[k].local = static_cast<int>(k);
    for (size_t k = 0; k < p.cols.size(); ++k) p.cols[k].local = static_cast<int>(k);
    return p;
}

static size_t n_items_max(int64_t n_obs, int64_t n_model, int nb) {
    return static_cast<size_t>((n_obs + 63) / 64 + (n_model + 63) / 64 + 2 * nb + 1);
}

struct SampleDims {
    const laue_geometry *geom;
    int64_t n_obs, n_model;
    int n_grains;
    int rho;                       // sparse assignment (0: dense)
};

// filter capacity per detected spot, in neighbours
constexpr int kCandPerNbr = 8;

struct SampleWs {
    double2 *part;
    float *F1;
    Col8 *colsE, *colsC;
    double *colHg;
    GeomF *geom;
    GrainF *grains;
    int *gflag;
    float *rmass, *cmass;
    double *obj;                   // objective partials (4 per work item) and totals
    Col8 *colsP;                   // previous E-step's columns and potentials (plan change)
    float *Fp, *Gp;
    int64_t *mboff;
    // sparse assignment (rho > 0)
    int *nbr = nullptr, *nbr_prev = nullptr, *cand_j = nullptr, *cand_n = nullptr, *knn_list = nullptr,
        *knn_nlist = nullptr;
    float *ncp = nullptr, *cand_c = nullptr, *col_cp = nullptr;
    int *col_row = nullptr, *knn_hist = nullptr;
    int *sk_in = nullptr, *sk_out = nullptr, *sv_in = nullptr, *sv_out = nullptr;
    void *sort_tmp = nullptr;
    size_t sort_tmp_bytes = 0;
    int64_t *col_off = nullptr, *oboff = nullptr;
};

struct BatchWs {
    SampleDesc *desc;
    SinkCtl *ctl;
    Item *rows, *cols;
    int2 *rows2, *cols2;      // workgroups of the two-per-lane tile shape
    int64_t *mbase, *gbase;
    CtlInit *init;
    ObjIn *objin;             // [2 n]: current and previous plan of each sample
};

static size_t carve_all(Carver &cv, BatchWs &bw, std::vector<SampleWs> &sw, const std::vector<SampleDims> &dims) {
    const int n = static_cast<int>(dims.size());
    size_t items = 0;
    for (const SampleDims &d : dims) items += n_items_max(d.n_obs, d.n_model, d.geom->n_rot * d.geom->n_det);
    bw.desc = cv.take<SampleDesc>(std::max(n, 1));
    bw.ctl = cv.take<SinkCtl>(std::max(n, 1));
    bw.rows = cv.take<Item>(std::max<size_t>(items, 1));
    bw.cols = cv.take<Item>(std::max<size_t>(items, 1));
    bw.rows2 = cv.take<int2>(std::max<size_t>(items, 1));
    bw.cols2 = cv.take<int2>(std::max<size_t>(items, 1));
    bw.mbase = cv.take<int64_t>(n + 1);
    bw.gbase = cv.take<int64_t>(n + 1);
    bw.init = cv.take<CtlInit>(std::max(n, 1));
    bw.objin = cv.take<ObjIn>(2 * std::max(n, 1));
    sw.resize(n);
    for (int s = 0; s < n; ++s) {
        const SampleDims &d = dims[s];
        const int nb = d.geom->n_rot * d.geom->n_det;
        SampleWs &w = sw[s];
        w.part = cv.take<double2>(n_items_max(d.n_obs, d.n_model, nb));
        w.obj = cv.take<double>(4 * n_items_max(d.n_obs, d.n_model, nb) + 8);
        w.F1 = cv.take<float>(std::max<int64_t>(d.n_obs, 1));
        w.colsE = cv.take<Col8>(std::max<int64_t>(d.n_model, 1));
        w.colsC = cv.take<Col8>(std::max<int64_t>(d.n_model, 1));
        w.colsP = cv.take<Col8>(std::max<int64_t>(d.n_model, 1));
        w.Fp = cv.take<float>(std::max<int64_t>(d.n_obs, 1));
        w.Gp = cv.take<float>(std::max<int64_t>(d.n_model, 1));
        w.colHg = cv.take<double>(std::max<int64_t>(d.n_model, 1) * kHg);
        w.geom = cv.take<GeomF>(1);
        w.grains = cv.take<GrainF>(std::max(d.n_grains, 1));
        w.gflag = cv.take<int>(std::max(d.n_grains, 1));
        w.rmass = cv.take<float>(std::max<int64_t>(d.n_obs, 1));
        w.cmass = cv.take<float>(std::max<int64_t>(d.n_model, 1));
        w.mboff = cv.take<int64_t>(nb + 1);
        if (d.rho > 0) {
            const int64_t no = std::max<int64_t>(d.n_obs, 1), nm = std::max<int64_t>(d.n_model, 1);
            const int64_t cap = static_cast<int64_t>(kCandPerNbr) * d.rho;
            w.nbr = cv.take<int>(no * d.rho);
            w.nbr_prev = cv.take<int>(no * d.rho);
            w.ncp = cv.take<float>(no * d.rho);
            w.cand_j = cv.take<int>(no * cap);
            w.cand_c = cv.take<float>(no * cap);
            w.cand_n = cv.take<int>(no);
            w.knn_list = cv.take<int>(no);
            w.knn_nlist = cv.take<int>(1);
            w.knn_hist = cv.take<int>(static_cast<int64_t>(nb) * kGrid * kGrid);
            w.sk_in = cv.take<int>(no * d.rho);
            w.sk_out = cv.take<int>(no * d.rho);
            w.sv_in = cv.take<int>(no * d.rho);
            w.sv_out = cv.take<int>(no * d.rho);
            // radix-sort scratch: a bound on what the sort asks for (its own
            // double buffers and digit histograms); checked at run time
            w.sort_tmp_bytes = static_cast<size_t>(no * d.rho) * 24 + (size_t(32) << 20);
            w.sort_tmp = cv.take<uint8_t>(static_cast<int64_t>(w.sort_tmp_bytes));
            w.col_off = cv.take<int64_t>(nm + 1);
            w.col_row = cv.take<int>(no * d.rho);
            w.col_cp = cv.take<float>(no * d.rho);
            w.oboff = cv.take<int64_t>(nb + 1);
        }
    }
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
    LAUE_REQUIRE(p->rho == 0 || p->rho == 8 || p->rho == 16 || p->rho == 32, LAUE_EINVAL,
                 "rho must be 0 (dense), 8, 16 or 32");
    LAUE_REQUIRE(p->outlier_model >= 0 && p->outlier_model <= 2, LAUE_EINVAL,
                 "outlier_model must be 0 (outlier row and column), 1 (unbalanced OT) or 2 (partial OT)");
    LAUE_REQUIRE(p->outlier_model != 2 || (std::isfinite(p->m_frac) && p->m_frac > 0 && p->m_frac <= 1),
                 LAUE_EINVAL, "partial OT needs 0 < m_frac <= 1");
    LAUE_REQUIRE(p->outlier_model != 1 || (std::isfinite(p->kappa) && p->kappa > 0 && std::isfinite(p->lam) &&
                                           p->lam > 0),
                 LAUE_EINVAL, "unbalanced OT needs finite kappa > 0 and lam > 0");
    return LAUE_OK;
}

// bin potentials a call reads: finite under the outlier row and column, unread
// under unbalanced OT
static bool bins_ok(const laue_ot_params *p, const laue_potentials *pot) {
    return p->outlier_model != 0 || (std::isfinite(pot->f0) && std::isfinite(pot->g0));
}

static int validate_gn(const laue_gn_params *gn) {
    LAUE_REQUIRE(gn && gn->k_gn >= 0 && std::isfinite(gn->mu_rel) && gn->mu_rel >= 0, LAUE_EINVAL,
                 "bad Gauss-Newton parameters");
    LAUE_REQUIRE(gn->method == 0 || gn->method == 1, LAUE_EINVAL,
                 "gn.method must be 0 (Gauss-Newton) or 1 (coordinate descent)");
    LAUE_REQUIRE(gn->method == 0 || (gn->k_newton >= 1 && gn->k_mm >= 1 && std::isfinite(gn->tol_x) &&
                                     gn->tol_x >= 0 && std::isfinite(gn->tol_r) && gn->tol_r >= 0),
                 LAUE_EINVAL, "coordinate descent needs k_newton >= 1, k_mm >= 1 and tolerances >= 0");
    return LAUE_OK;
}

static int validate_em_params(const laue_em_params *par) {
    int rc;
    LAUE_REQUIRE(par != nullptr, LAUE_EINVAL, "EM parameters are NULL");
    if ((rc = validate_ot(&par->ot, false))) return rc;
    LAUE_REQUIRE(std::isfinite(par->eps_start) && std::isfinite(par->eps_end) && par->eps_start > 0 &&
                     par->eps_end > 0,
                 LAUE_EINVAL, "bad temperature schedule");
    LAUE_REQUIRE(std::isfinite(par->eps_cool) && par->eps_cool >= 0.0 && par->eps_cool < 1.0, LAUE_EINVAL,
                 "eps_cool must be 0 (stage schedule) or in (0, 1)");
    if (par->eps_cool > 0.0) {
        LAUE_REQUIRE(std::log(par->eps_start / par->eps_end) / -std::log(par->eps_cool) < 100000.0, LAUE_EINVAL,
                     "the cooling schedule has more than 100000 temperatures");
        LAUE_REQUIRE(par->final_iters >= 0 && std::isfinite(par->zeta_tol), LAUE_EINVAL,
                     "final_iters must be >= 0 and zeta_tol finite");
    } else {
        LAUE_REQUIRE(par->n_stages >= 1 && par->iters_per_stage >= 1, LAUE_EINVAL, "bad temperature schedule");
    }
    LAUE_REQUIRE(std::isfinite(par->sigma_mm) && par->sigma_mm >= 0.0, LAUE_EINVAL, "sigma_mm must be >= 0");
    if ((rc = validate_gn(&par->gn))) return rc;
    LAUE_REQUIRE(par->launch >= 0 && par->launch <= 2, LAUE_EINVAL, "launch must be 0, 1 or 2");
    LAUE_REQUIRE(par->tile >= 0 && par->tile <= 2, LAUE_EINVAL, "tile must be 0, 1 or 2");
    return LAUE_OK;
}

// ---------------------------------------------------------------- plan summaries

// Sums of the plan Q = exp((f + g - c)/eps) with its bins (Eqs. elbo,
// estep_obj): per 64-row item, lane = detected spot, over its block's model
// spots (or its neighbours under the sparse assignment) and its outlier entry
// q_i0: mass, <c, Q> over the matches, the outlier entries' cost and
// sum Q ln Q; per 64-column item the unmatched entries q_0j.  Each item's
// four sums go to the sample's obj[4 item + k] (column items after the row
// items); k_obj_final adds them in item order, one workgroup per sample, and
// writes the totals (mass, <c,Q> matches, total cost, sum Q ln Q) after them.
__global__ __launch_bounds__(64) void k_obj_rows(const Item *__restrict__ items, const SampleDesc *__restrict__ descs,
                                                 const ObjIn *__restrict__ oin) {
    const Item it = items[blockIdx.x];
    const SampleDesc &D = descs[it.s];
    const ObjIn A = oin[it.s];
    const SinkParams p = D.sp;
    const double kexp = 1.4426950408889634 / A.eps;
    const float kx = static_cast<float>(kexp);
    const float K = p.twoD2 * kx;
    const int i = it.r0 + static_cast<int>(threadIdx.x);
    const bool act = i < it.r1;
    const float p1 = act ? D.p1[i] : 0.0f, p2 = act ? D.p2[i] : 0.0f, f = act ? D.f[i] : 0.0f;
    const float fk = f * kx;
    double m = 0.0, cin = 0.0, cb = 0.0, ql = 0.0;
    float am = 0.0f, ac = 0.0f, al = 0.0f;
    if (act) {
        if (D.rho > 0) {
            for (int q = 0; q < D.rho; ++q) {
                const int j = D.nbr[q * D.n_obs + i];
                if (j < 0) continue;
                const float cp = D.ncp[q * D.n_obs + i];
                const float e = fmaf(-K, cp, fmaf(D.g[j], kx, fk));
                const float Q = fast_exp2(e);
                if (Q > 0.0f) {
                    am += Q;
                    ac = fmaf(Q, p.twoD2 * cp, ac);
                    al = fmaf(Q, e, al);
                }
            }
        } else {
            for (int j = it.c0; j < it.c1; ++j) {
                const Col8 c = D.colsE[j];
                const float cp = chord_cp(p1, p2, c.s1, c.s2, c.v1, c.v2, c.vv, c.vv2);
                const float e = fmaf(-K, cp, fmaf(D.g[j], kx, fk));
                const float Q = fast_exp2(e);
                if (Q > 0.0f) {
                    am += Q;
                    ac = fmaf(Q, p.twoD2 * cp, ac);
                    al = fmaf(Q, e, al);
                }
            }
        }
        m = static_cast<double>(am);
        cin = static_cast<double>(ac);
        ql = static_cast<double>(al) * 0.6931471805599453;   // e is in log2 units
        const double lb = (static_cast<double>(f) + A.g0 - p.c_out) / A.eps;
        const double qb = exp(lb);
        if (qb > 0.0) {
            m += qb;
            cb = p.c_out * qb;
            ql += qb * lb;
        }
    }
    m = wave_sum(m);
    cin = wave_sum(cin);
    cb = wave_sum(cb);
    ql = wave_sum(ql);
    if (threadIdx.x == 0) {
        double *o = D.obj + 4 * static_cast<int64_t>(it.local);
        o[0] = m;
        o[1] = cin;
        o[2] = cb;
        o[3] = ql;
    }
}

__global__ __launch_bounds__(64) void k_obj_cols(const Item *__restrict__ items, const SampleDesc *__restrict__ descs,
                                                 const ObjIn *__restrict__ oin) {
    const Item it = items[blockIdx.x];
    const SampleDesc &D = descs[it.s];
    const ObjIn A = oin[it.s];
    const SinkParams p = D.sp;
    const int j = it.c0 + static_cast<int>(threadIdx.x);
    double m = 0.0, cb = 0.0, ql = 0.0;
    if (j < it.c1) {
        const double lb = (A.f0 + static_cast<double>(D.g[j]) - p.c_unm) / A.eps;
        const double qb = exp(lb);
        if (qb > 0.0) {
            m = qb;
            cb = p.c_unm * qb;
            ql = qb * lb;
        }
    }
    m = wave_sum(m);
    cb = wave_sum(cb);
    ql = wave_sum(ql);
    if (threadIdx.x == 0) {
        double *o = D.obj + 4 * (static_cast<int64_t>(D.n_row_items) + it.local);
        o[0] = m;
        o[1] = 0.0;
        o[2] = cb;
        o[3] = ql;
    }
}

__global__ __launch_bounds__(64) void k_obj_final(const SampleDesc *__restrict__ descs,
                                                  const ObjIn *__restrict__ oin) {
    const SampleDesc &D = descs[blockIdx.x];
    const ObjIn A = oin[blockIdx.x];
    const int n = D.n_row_items + D.n_col_items;
    double t[4] = {0.0, 0.0, 0.0, 0.0};
    for (int w = threadIdx.x; w < n; w += 64)
        for (int k = 0; k < 4; ++k) t[k] += D.obj[4 * static_cast<int64_t>(w) + k];
    for (int k = 0; k < 4; ++k) t[k] = wave_sum(t[k]);
    if (threadIdx.x != 0) return;
    const SinkParams p = D.sp;
    double mass = t[0], cin = t[1], ctot = t[1] + t[2], ql = t[3];
    const double l00 = (A.f0 + A.g0 - p.c_sink) / A.eps;
    const double q00 = exp(l00);
    if (q00 > 0.0) {
        mass += q00;
        ctot += p.c_sink * q00;
        ql += q00 * l00;
    }
    double *o = D.obj + 4 * static_cast<int64_t>(n);
    o[0] = mass;
    o[1] = cin;
    o[2] = ctot;
    o[3] = ql;
}

// Q_0j = exp((f0 + g_j - c_unm)/eps) of every model spot into the assignment
// output (0 without bins).  One block row per sample (blockIdx.y).
__global__ void k_assign_unm(const SampleDesc *__restrict__ descs, const ObjIn *__restrict__ oin) {
    const SampleDesc &D = descs[blockIdx.y];
    if (!D.qunm) return;
    const int64_t j = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (j >= D.n_model) return;
    const ObjIn A = oin[blockIdx.y];
    D.qunm[j] = static_cast<float>(exp((A.f0 + static_cast<double>(D.g[j]) - D.sp.c_unm) / A.eps));
}

// Plan change zeta^2 = ||Q - Q'||_F^2 between the current plan (f, g,
// columns colsE, oin[s]) and the previous E-step's (fprev, gprev, colsP,
// oin[n + s]), dense assignment: per 64-row item, lane = detected spot, the
// squared differences over its block's model spots (entries evaluated in
// FP32 as in the passes, squares summed in FP32 over the block, then FP64)
// plus its outlier entry; per 64-column item the unmatched entries; partials
// into obj[4 item] and the corner entry in k_dq_final.
__global__ __launch_bounds__(64) void k_dq_rows(const Item *__restrict__ items, const SampleDesc *__restrict__ descs,
                                                const ObjIn *__restrict__ oin, int n) {
    const Item it = items[blockIdx.x];
    const SampleDesc &D = descs[it.s];
    const ObjIn A = oin[it.s], B = oin[n + it.s];
    const SinkParams p = D.sp;
    const float ka = static_cast<float>(1.4426950408889634 / A.eps);
    const float kb = static_cast<float>(1.4426950408889634 / B.eps);
    const float Ka = p.twoD2 * ka, Kb = p.twoD2 * kb;
    const int i = it.r0 + static_cast<int>(threadIdx.x);
    const bool act = i < it.r1;
    double s = 0.0;
    if (act) {
        const float p1 = D.p1[i], p2 = D.p2[i];
        const float fa = D.f[i] * ka, fb = D.fprev[i] * kb;
        float acc = 0.0f;
        for (int j = it.c0; j < it.c1; ++j) {
            const Col8 c = D.colsE[j];
            const Col8 d = D.colsP[j];
            const float qa = fast_exp2(fmaf(-Ka, chord_cp(p1, p2, c.s1, c.s2, c.v1, c.v2, c.vv, c.vv2),
                                            fmaf(D.g[j], ka, fa)));
            const float qb = fast_exp2(fmaf(-Kb, chord_cp(p1, p2, d.s1, d.s2, d.v1, d.v2, d.vv, d.vv2),
                                            fmaf(D.gprev[j], kb, fb)));
            const float dq = qa - qb;
            acc = fmaf(dq, dq, acc);
        }
        const double ba = exp((static_cast<double>(D.f[i]) + A.g0 - p.c_out) / A.eps);
        const double bb = exp((static_cast<double>(D.fprev[i]) + B.g0 - p.c_out) / B.eps);
        s = static_cast<double>(acc) + (ba - bb) * (ba - bb);
    }
    s = wave_sum(s);
    if (threadIdx.x == 0) D.obj[4 * static_cast<int64_t>(it.local)] = s;
}

// The same for the sparse assignment (rho > 0): a detected spot's entries
// are those of its rho neighbours in the current plan (nbr) and of its
// neighbours of the previous E-step in the previous one (nbr_prev, -1 for an
// empty slot); an entry in one set only counts with 0 from the other plan
// (the plans are 0 off their neighbour sets).  Both lists in registers.
constexpr int kMaxRho = 32;
__global__ __launch_bounds__(64) void k_dq_rows_sparse(const Item *__restrict__ items,
                                                       const SampleDesc *__restrict__ descs,
                                                       const ObjIn *__restrict__ oin, int n) {
    const Item it = items[blockIdx.x];
    const SampleDesc &D = descs[it.s];
    const ObjIn A = oin[it.s], B = oin[n + it.s];
    const SinkParams p = D.sp;
    const float ka = static_cast<float>(1.4426950408889634 / A.eps);
    const float kb = static_cast<float>(1.4426950408889634 / B.eps);
    const float Ka = p.twoD2 * ka, Kb = p.twoD2 * kb;
    const int i = it.r0 + static_cast<int>(threadIdx.x);
    const bool act = i < it.r1;
    const int rho = min(D.rho, kMaxRho);
    double s = 0.0;
    if (act) {
        const float p1 = D.p1[i], p2 = D.p2[i];
        const float fa = D.f[i] * ka, fb = D.fprev[i] * kb;
        int na[kMaxRho], nb[kMaxRho];
#pragma unroll
        for (int q = 0; q < kMaxRho; ++q) {
            na[q] = q < rho ? D.nbr[static_cast<int64_t>(q) * D.n_obs + i] : -1;
            nb[q] = q < rho ? D.nbr_prev[static_cast<int64_t>(q) * D.n_obs + i] : -1;
        }
        float acc = 0.0f;
#pragma unroll
        for (int q = 0; q < kMaxRho; ++q) {
            const int j = na[q];
            if (j < 0) continue;
            const Col8 c = D.colsE[j];
            const float qa = fast_exp2(fmaf(-Ka, chord_cp(p1, p2, c.s1, c.s2, c.v1, c.v2, c.vv, c.vv2),
                                            fmaf(D.g[j], ka, fa)));
            bool both = false;
#pragma unroll
            for (int r = 0; r < kMaxRho; ++r) both = both || nb[r] == j;
            float qb = 0.0f;
            if (both) {
                const Col8 d = D.colsP[j];
                qb = fast_exp2(fmaf(-Kb, chord_cp(p1, p2, d.s1, d.s2, d.v1, d.v2, d.vv, d.vv2),
                                    fmaf(D.gprev[j], kb, fb)));
            }
            const float dq = qa - qb;
            acc = fmaf(dq, dq, acc);
        }
#pragma unroll
        for (int r = 0; r < kMaxRho; ++r) {
            const int j = nb[r];
            if (j < 0) continue;
            bool both = false;
#pragma unroll
            for (int q = 0; q < kMaxRho; ++q) both = both || na[q] == j;
            if (both) continue;
            const Col8 d = D.colsP[j];
            const float qb = fast_exp2(fmaf(-Kb, chord_cp(p1, p2, d.s1, d.s2, d.v1, d.v2, d.vv, d.vv2),
                                            fmaf(D.gprev[j], kb, fb)));
            acc = fmaf(qb, qb, acc);
        }
        const double ba = exp((static_cast<double>(D.f[i]) + A.g0 - p.c_out) / A.eps);
        const double bb = exp((static_cast<double>(D.fprev[i]) + B.g0 - p.c_out) / B.eps);
        s = static_cast<double>(acc) + (ba - bb) * (ba - bb);
    }
    s = wave_sum(s);
    if (threadIdx.x == 0) D.obj[4 * static_cast<int64_t>(it.local)] = s;
}

__global__ __launch_bounds__(64) void k_dq_cols(const Item *__restrict__ items, const SampleDesc *__restrict__ descs,
                                                const ObjIn *__restrict__ oin, int n) {
    const Item it = items[blockIdx.x];
    const SampleDesc &D = descs[it.s];
    const ObjIn A = oin[it.s], B = oin[n + it.s];
    const int j = it.c0 + static_cast<int>(threadIdx.x);
    double s = 0.0;
    if (j < it.c1) {
        const double ua = exp((A.f0 + static_cast<double>(D.g[j]) - D.sp.c_unm) / A.eps);
        const double ub = exp((B.f0 + static_cast<double>(D.gprev[j]) - D.sp.c_unm) / B.eps);
        s = (ua - ub) * (ua - ub);
    }
    s = wave_sum(s);
    if (threadIdx.x == 0) D.obj[4 * (static_cast<int64_t>(D.n_row_items) + it.local)] = s;
}

// zeta of each sample (one workgroup per sample) into obj[4 n_items]
__global__ __launch_bounds__(64) void k_dq_final(const SampleDesc *__restrict__ descs, const ObjIn *__restrict__ oin,
                                                 int n) {
    const SampleDesc &D = descs[blockIdx.x];
    const ObjIn A = oin[blockIdx.x], B = oin[n + blockIdx.x];
    const int m = D.n_row_items + D.n_col_items;
    double t = 0.0;
    for (int w = threadIdx.x; w < m; w += 64) t += D.obj[4 * static_cast<int64_t>(w)];
    t = wave_sum(t);
    if (threadIdx.x != 0) return;
    const double a = exp((A.f0 + A.g0 - D.sp.c_sink) / A.eps), b = exp((B.f0 + B.g0 - D.sp.c_sink) / B.eps);
    D.obj[4 * static_cast<int64_t>(m)] = sqrt(t + (a - b) * (a - b));
}

// One sample's inputs to the engine.
struct SampleIn {
    const laue_geometry *geom;
    const laue_planes *planes;     // may be NULL (Sinkhorn only)
    const laue_obs_spots *obs;
    laue_model_spots *model;
    const laue_ot_params *ot;
    laue_grains *grains;           // may be NULL (Sinkhorn only)
    laue_potentials *pot;
    double mu_rel;
    laue_assignments *assign;      // may be NULL
    double *step_norm;             // may be NULL
    const laue_gn_params *gn;      // may be NULL (Gauss-Newton)
};

// E- and M-steps of one or more samples on one stream: one launch per pass.
struct BatchEngine {
    hipStream_t s = nullptr;
    int n = 0;
    BatchWs bw{};
    std::vector<SampleWs> sw;
    std::vector<SampleIn> in;
    std::vector<SampleDesc> hd;
    std::vector<SamplePlan> plans;
    std::vector<int64_t> mbase, gbase;
    int n_rows = 0, n_cols = 0, n_rows2 = 0, n_cols2 = 0;
    int rho = 0;                                 // sparse assignment (0: dense)
    int mmethod = 0, k_newton = 1;               // M-step: 0 Gauss-Newton, 1 the paper's coordinate descent
    std::vector<int64_t> sparse_entries;         // per sample: kept pairs of the current sets
    // per sample: streamed entries, Sinkhorn passes and their entries, M-step entries
    std::vector<int64_t> entries, passes, pass_entries, m_entries;
    std::vector<SinkCtl> hctl;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    double sink_ms = 0.0, mstep_ms = 0.0;
    // issuing of the Sinkhorn passes: 1 direct launches, 2 graph replay, 0 tune
    int launch_mode = 1, chosen = 0, polls = 0;
    double t_direct = -1.0, t_graph = -1.0;     // ms per iteration on chunks where every pass worked
    std::vector<std::pair<int, hipGraphExec_t>> graphs;   // one captured chunk per chunk length
    hipGraphExec_t mgraph = nullptr;            // captured M-step + forward evaluation
    int mgraph_kgn = -1;
    hipStream_t cap_stream = nullptr;
    std::vector<int> stage_iters;               // iterations of the latest Sinkhorn of each stage
    // tile shape (1 or 2 rows / columns per lane): fixed, or tuned per stage
    // on the first row + column pass of a Sinkhorn (which always works)
    int tile_mode = 1;
    std::vector<int> stage_tile;
    std::vector<int> tiles_used;
    hipEvent_t tev[6] = {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
    // false: no HIP events (no timing); direct launches and a fixed tile shape
    // then create no HIP object at all
    bool timing = true;

    ~BatchEngine() {
        if (!graphs.empty()) (void)hipStreamSynchronize(s);
        if (mgraph) (void)hipStreamSynchronize(s);
        for (auto &g : graphs) (void)hipGraphExecDestroy(g.second);
        if (mgraph) (void)hipGraphExecDestroy(mgraph);
        if (cap_stream) (void)hipStreamDestroy(cap_stream);
        if (ev0) (void)hipEventDestroy(ev0);
        if (ev1) (void)hipEventDestroy(ev1);
        for (auto e : tev)
            if (e) (void)hipEventDestroy(e);
    }

    // A captured graph of `chunk` Sinkhorn iterations (row and column pass of
    // every sample); the passes read their state from the control blocks, so
    // one graph serves every chunk, temperature and EM iteration of the call.
    // one row pass and one column pass in tile shape R (empty grids skipped)
    void row_launch(hipStream_t st, int R) {
        if (rho > 0) {
            if (n_rows) k_row_sparse<<<n_rows, 64, 0, st>>>(bw.rows, bw.desc);
            return;
        }
        if (R == 2 && n_rows2) k_row<2><<<n_rows2, 64, 0, st>>>(bw.rows, bw.rows2, bw.desc);
        if (R == 1 && n_rows) k_row<1><<<n_rows, 64, 0, st>>>(bw.rows, bw.rows2, bw.desc);
    }
    void col_launch(hipStream_t st, int R) {
        if (rho > 0) {
            if (n_cols) k_col_sparse<<<n_cols, 64, 0, st>>>(bw.cols, bw.desc);
            return;
        }
        if (R == 2 && n_cols2) k_col<2><<<n_cols2, 64, 0, st>>>(bw.cols, bw.cols2, bw.desc);
        if (R == 1 && n_cols) k_col<1><<<n_cols, 64, 0, st>>>(bw.cols, bw.cols2, bw.desc);
    }

    // The neighbour sets of every sample from its packed E-step columns
    // (colsE), and their column lists.
    int build_neighbors() {
        if (rho <= 0) return LAUE_OK;
        for (int k = 0; k < n; ++k) {
            k_zero_i<<<1, 64, 0, s>>>(sw[k].knn_nlist, 1);
            const int64_t nm = std::max<int64_t>(in[k].model->n, 1);
            const int64_t nh = static_cast<int64_t>(in[k].geom->n_rot) * in[k].geom->n_det * kGrid * kGrid;
            k_zero_i<<<static_cast<unsigned>((nh + 255) / 256), 256, 0, s>>>(sw[k].knn_hist, nh);
            if (in[k].model->n > 0)
                k_knn_hist<<<static_cast<unsigned>((in[k].model->n + 255) / 256), 256, 0, s>>>(bw.desc, k);
        }
        if (n_rows) {
            k_knn_filter<<<n_rows, 64, 0, s>>>(bw.rows, bw.desc);
            if (rho == 8) k_knn_select<8><<<n_rows, 64, 0, s>>>(bw.rows, bw.desc);
            if (rho == 16) k_knn_select<16><<<n_rows, 64, 0, s>>>(bw.rows, bw.desc);
            if (rho == 32) k_knn_select<32><<<n_rows, 64, 0, s>>>(bw.rows, bw.desc);
        }
        LAUE_CHECK_HIP(hipGetLastError());
        std::vector<int> nl(n, 0);
        for (int k = 0; k < n; ++k)
            LAUE_CHECK_HIP(hipMemcpyAsync(&nl[k], sw[k].knn_nlist, sizeof(int), hipMemcpyDeviceToHost, s));
        LAUE_CHECK_HIP(hipStreamSynchronize(s));
        sparse_entries.assign(n, 0);
        for (int k = 0; k < n; ++k) {
            const int64_t no = in[k].obs->n, nm = in[k].model->n;
            if (nl[k] > 0) {
                const unsigned g = static_cast<unsigned>((nl[k] + 63) / 64);
                if (rho == 8) k_knn_exact<8><<<g, 64, 0, s>>>(bw.desc, k, nl[k]);
                if (rho == 16) k_knn_exact<16><<<g, 64, 0, s>>>(bw.desc, k, nl[k]);
                if (rho == 32) k_knn_exact<32><<<g, 64, 0, s>>>(bw.desc, k, nl[k]);
            }
            if (no == 0 || nm == 0) {
                // no pairs: every column list is empty
                if (nm > 0) {
                    const int64_t w = 2 * (nm + 1);   // int64 offsets as int words
                    k_zero_i<<<static_cast<unsigned>((w + 255) / 256), 256, 0, s>>>(
                        reinterpret_cast<int *>(sw[k].col_off), w);
                }
                continue;
            }
            const int64_t ne = no * rho;
            k_knn_keys<<<static_cast<unsigned>((ne + 255) / 256), 256, 0, s>>>(bw.desc, k);
            int bits = 1;
            while ((int64_t(1) << bits) <= nm) ++bits;
            size_t tmp = 0;
            LAUE_CHECK_HIP(hipcub::DeviceRadixSort::SortPairs(nullptr, tmp, sw[k].sk_in, sw[k].sk_out, sw[k].sv_in,
                                                             sw[k].sv_out, static_cast<int>(ne), 0, bits, s));
            LAUE_REQUIRE(tmp <= sw[k].sort_tmp_bytes, LAUE_EWORKSPACE,
                         "internal: radix sort needs " + std::to_string(tmp) + " bytes, the workspace holds " +
                             std::to_string(sw[k].sort_tmp_bytes));
            LAUE_CHECK_HIP(hipcub::DeviceRadixSort::SortPairs(sw[k].sort_tmp, tmp, sw[k].sk_in, sw[k].sk_out,
                                                             sw[k].sv_in, sw[k].sv_out, static_cast<int>(ne), 0,
                                                             bits, s));
            k_knn_offsets<<<static_cast<unsigned>((nm + 1 + 255) / 256), 256, 0, s>>>(bw.desc, k, sw[k].sk_out);
            k_knn_gather<<<static_cast<unsigned>((ne + 255) / 256), 256, 0, s>>>(bw.desc, k);
        }
        LAUE_CHECK_HIP(hipGetLastError());
        std::vector<int64_t> tot(n, 0);
        for (int k = 0; k < n; ++k)
            if (in[k].model->n > 0 && in[k].obs->n > 0)
                LAUE_CHECK_HIP(hipMemcpyAsync(&tot[k], sw[k].col_off + in[k].model->n, sizeof(int64_t),
                                              hipMemcpyDeviceToHost, s));
        LAUE_CHECK_HIP(hipStreamSynchronize(s));
        sparse_entries = tot;
        return LAUE_OK;
    }

    // entries one pass streams for sample k
    int64_t pass_work(int k) const { return rho > 0 ? sparse_entries[k] : plans[k].entries; }
    void pass_pair(hipStream_t st, int R) {
        row_launch(st, R);
        col_launch(st, R);
    }

    int graph_for(int chunk, int R, hipGraphExec_t *out) {
        const int key = 4 * chunk + R;
        for (auto &g : graphs)
            if (g.first == key) {
                *out = g.second;
                return LAUE_OK;
            }
        if (!cap_stream) LAUE_CHECK_HIP(hipStreamCreateWithFlags(&cap_stream, hipStreamNonBlocking));
        LAUE_CHECK_HIP(hipStreamBeginCapture(cap_stream, hipStreamCaptureModeThreadLocal));
        for (int c = 0; c < chunk; ++c) pass_pair(cap_stream, R);
        const hipError_t le = hipGetLastError();
        hipGraph_t g = nullptr;
        const hipError_t ce = hipStreamEndCapture(cap_stream, &g);
        LAUE_CHECK_HIP(le);
        LAUE_CHECK_HIP(ce);
        hipGraphExec_t x = nullptr;
        const hipError_t ie = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        LAUE_CHECK_HIP(ie);
        graphs.emplace_back(key, x);
        *out = x;
        return LAUE_OK;
    }

    int mstep_graph(int k_gn, hipGraphExec_t *out) {
        if (mgraph && mgraph_kgn == k_gn) {
            *out = mgraph;
            return LAUE_OK;
        }
        if (mgraph) {
            LAUE_CHECK_HIP(hipStreamSynchronize(s));
            (void)hipGraphExecDestroy(mgraph);
            mgraph = nullptr;
        }
        if (!cap_stream) LAUE_CHECK_HIP(hipStreamCreateWithFlags(&cap_stream, hipStreamNonBlocking));
        LAUE_CHECK_HIP(hipStreamBeginCapture(cap_stream, hipStreamCaptureModeThreadLocal));
        mstep_launches(cap_stream, k_gn);
        const hipError_t le = hipGetLastError();
        hipGraph_t g = nullptr;
        const hipError_t ce = hipStreamEndCapture(cap_stream, &g);
        LAUE_CHECK_HIP(le);
        LAUE_CHECK_HIP(ce);
        const hipError_t ie = hipGraphInstantiate(&mgraph, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        LAUE_CHECK_HIP(ie);
        mgraph_kgn = k_gn;
        *out = mgraph;
        return LAUE_OK;
    }

    int timer_start() {
        if (!timing) return LAUE_OK;
        if (!ev0) {
            LAUE_CHECK_HIP(hipEventCreate(&ev0));
            LAUE_CHECK_HIP(hipEventCreate(&ev1));
        }
        LAUE_CHECK_HIP(hipEventRecord(ev0, s));
        return LAUE_OK;
    }

    int timer_stop(double *acc, double *dt = nullptr) {
        if (!timing) {
            if (dt) *dt = 0.0;
            return LAUE_OK;
        }
        LAUE_CHECK_HIP(hipEventRecord(ev1, s));
        LAUE_CHECK_HIP(hipEventSynchronize(ev1));
        float ms = 0.0f;
        LAUE_CHECK_HIP(hipEventElapsedTime(&ms, ev0, ev1));
        *acc += ms;
        if (dt) *dt = ms;
        return LAUE_OK;
    }

    int setup(const std::vector<SampleIn> &samples, void *ws, size_t ws_bytes, void *stream, bool need_geo) {
        int rc;
        in = samples;
        n = static_cast<int>(in.size());
        std::vector<SampleDims> dims(n);
        for (int k = 0; k < n; ++k) {
            const SampleIn &a = in[k];
            if ((rc = validate_geometry(a.geom))) return rc;
            const int nb = a.geom->n_rot * a.geom->n_det;
            if ((rc = validate_obs(a.obs, nb)) || (rc = validate_model(a.model, nb, need_geo))) return rc;
            const double t_a = a.ot->t_b + static_cast<double>(a.obs->n) - static_cast<double>(a.model->n);
            LAUE_REQUIRE(a.ot->outlier_model != 0 || t_a >= 0, LAUE_EINFEASIBLE,
                         "infeasible masses: T_a = T_b + |I| - |J| = " + std::to_string(t_a) + " < 0");
            LAUE_REQUIRE(a.pot != nullptr, LAUE_EINVAL, "potentials are NULL");
            LAUE_REQUIRE(a.obs->n == 0 || a.pot->f, LAUE_EINVAL, "f is NULL");
            LAUE_REQUIRE(a.model->n == 0 || a.pot->g, LAUE_EINVAL, "g is NULL");
            LAUE_REQUIRE(a.ot->rho == in[0].ot->rho, LAUE_EINVAL, "samples of a batch share rho");
            LAUE_REQUIRE(static_cast<double>(a.obs->n) * std::max(a.ot->rho, 1) < 2147483647.0, LAUE_EINVAL,
                         "too many detected spots for sparse lists");
            dims[k] = SampleDims{a.geom, a.obs->n, a.model->n, a.grains ? a.grains->n : 0, a.ot->rho};
        }
        rho = n > 0 ? in[0].ot->rho : 0;
        mmethod = n > 0 && in[0].gn ? in[0].gn->method : 0;
        k_newton = n > 0 && in[0].gn ? std::max(in[0].gn->k_newton, 1) : 1;
        for (int k = 0; k < n; ++k) {
            const laue_gn_params *gk = in[k].gn;
            LAUE_REQUIRE((gk ? gk->method : 0) == mmethod && (mmethod == 0 || gk->k_newton == k_newton), LAUE_EINVAL,
                         "samples of a batch share gn.method and gn.k_newton");
            LAUE_REQUIRE(mmethod == 0 || !in[k].planes || in[k].planes->n <= kMaxPlanesMM, LAUE_EINVAL,
                         "the coordinate-descent M-step holds at most 1024 planes");
        }
        Carver cv(ws);
        const size_t need = carve_all(cv, bw, sw, dims);
        if ((rc = check_ws(ws, ws_bytes, need))) return rc;
        s = static_cast<hipStream_t>(stream);
        std::vector<Item> rows, cols;
        hd.assign(n, SampleDesc{});
        plans.resize(n);
        mbase.assign(n + 1, 0);
        gbase.assign(n + 1, 0);
        entries.assign(n, 0);
        passes.assign(n, 0);
        pass_entries.assign(n, 0);
        m_entries.assign(n, 0);
        for (int k = 0; k < n; ++k) {
            const SampleIn &a = in[k];
            const int nb = a.geom->n_rot * a.geom->n_det;
            plans[k] = make_plan(a.obs->block_off, a.model->block_off, nb, k);
            rows.insert(rows.end(), plans[k].rows.begin(), plans[k].rows.end());
            cols.insert(cols.end(), plans[k].cols.begin(), plans[k].cols.end());
            SampleDesc &D = hd[k];
            D.p1 = a.obs->p1;
            D.p2 = a.obs->p2;
            D.f = a.pot->f;
            D.f1 = sw[k].F1;
            D.g = a.pot->g;
            D.colsE = sw[k].colsE;
            D.colsC = sw[k].colsC;
            D.ctl = bw.ctl + k;
            D.part = sw[k].part;
            D.n_row_items = static_cast<int>(plans[k].rows.size());
            D.n_col_items = static_cast<int>(plans[k].cols.size());
            SinkParams &sp = D.sp;
            sp.c_out = a.ot->c_out;
            sp.c_unm = a.ot->c_unm;
            sp.c_sink = a.ot->c_sink;
            sp.unb = a.ot->outlier_model == 1 ? 1 : 0;
            sp.part = a.ot->outlier_model == 2 ? 1 : 0;
            // no bins under unbalanced or partial OT: zero masses make their potentials -inf
            const bool nobins = sp.unb || sp.part;
            sp.t_b = nobins ? 0.0 : a.ot->t_b;
            sp.t_a = nobins ? 0.0 : a.ot->t_b + static_cast<double>(a.obs->n) - static_cast<double>(a.model->n);
            sp.kappa = sp.unb ? a.ot->kappa : 0.0;
            sp.lam = sp.unb ? a.ot->lam : 0.0;
            // partial OT: m = m_frac * sum_b min(|I_b|, |J_b|), the most the block plans can carry
            double mmax = 0.0;
            for (int b = 0; b < nb; ++b)
                mmax += static_cast<double>(std::min(a.obs->block_off[b + 1] - a.obs->block_off[b],
                                                     a.model->block_off[b + 1] - a.model->block_off[b]));
            sp.mass = sp.part ? a.ot->m_frac * mmax : 0.0;
            sp.tol = a.ot->tol;
            sp.twoD2 = static_cast<float>(2.0 * a.ot->distance * a.ot->distance);
            sp.n_max = a.ot->n_max;
            D.mplane = a.model->plane;
            D.mgrain = a.model->grain;
            D.mblock = a.model->block;
            D.s1 = a.model->s1;
            D.s2 = a.model->s2;
            D.vn = a.model->vn;
            D.v1 = a.model->v1;
            D.v2 = a.model->v2;
            D.lam = a.model->lam;
            D.mboff = sw[k].mboff;
            D.n_obs = a.obs->n;
            D.n_model = a.model->n;
            D.nb = nb;
            D.n_grains = a.grains ? a.grains->n : 0;
            D.n_planes = a.planes ? a.planes->n : 0;
            D.geom = sw[k].geom;
            D.grains = sw[k].grains;
            D.q = a.grains ? a.grains->q : nullptr;
            D.x = a.grains ? a.grains->x : nullptr;
            D.colHg = sw[k].colHg;
            D.step_norm = a.step_norm;
            D.W = a.planes ? a.planes->w : nullptr;
            D.Dsp = a.planes ? a.planes->d : nullptr;
            D.D2 = a.ot->distance * a.ot->distance;
            D.mu_rel = a.mu_rel;
            D.gflag = sw[k].gflag;
            D.rmass = sw[k].rmass;
            D.cmass = sw[k].cmass;
            D.k_mm = a.gn ? a.gn->k_mm : 1;
            D.tol_x = a.gn ? a.gn->tol_x : 0.0;
            D.tol_r = a.gn ? a.gn->tol_r : 0.0;
            D.obj = sw[k].obj;
            D.colsP = sw[k].colsP;
            D.fprev = sw[k].Fp;
            D.gprev = sw[k].Gp;
            if (a.assign && a.assign->q_unm) D.qunm = a.assign->q_unm;
            if (a.assign && a.assign->j_star && a.assign->grain && a.assign->q_star && a.assign->q_out) {
                D.jstar = a.assign->j_star;
                D.gstar = a.assign->grain;
                D.qstar = a.assign->q_star;
                D.qout = a.assign->q_out;
            }
            if (rho > 0) {
                D.rho = rho;
                D.cand_cap = kCandPerNbr * rho;
                // filter threshold: 3 rho model spots expected within it for a
                // uniform block (in-plane radius r with pi r^2 n_b / l^2 = 3 rho,
                // c' ~ r^2 / (2 D^2) near normal incidence)
                double area = 0.0;
                for (int d = 0; d < a.geom->n_det; ++d)
                    area = std::max(area, 4.0 * a.geom->det[d].half_size * a.geom->det[d].half_size);
                D.knn_k = static_cast<float>(3.0 * rho * area / (M_PI * 2.0 * a.ot->distance * a.ot->distance));
                D.nbr = sw[k].nbr;
                D.nbr_prev = sw[k].nbr_prev;
                D.ncp = sw[k].ncp;
                D.cand_j = sw[k].cand_j;
                D.cand_c = sw[k].cand_c;
                D.cand_n = sw[k].cand_n;
                D.knn_list = sw[k].knn_list;
                D.knn_nlist = sw[k].knn_nlist;
                D.knn_hist = sw[k].knn_hist;
                D.sort_key = sw[k].sk_in;
                D.sort_val = sw[k].sv_in;
                D.sorted_val = sw[k].sv_out;
                D.col_off = sw[k].col_off;
                D.col_row = sw[k].col_row;
                D.col_cp = sw[k].col_cp;
                D.oboff = sw[k].oboff;
                LAUE_CHECK_HIP(hipMemcpyAsync(sw[k].oboff, a.obs->block_off, (nb + 1) * sizeof(int64_t),
                                              hipMemcpyHostToDevice, s));
            }
            mbase[k + 1] = mbase[k] + a.model->n;
            gbase[k + 1] = gbase[k] + D.n_grains;
            GeomF hg;
            make_geomf(a.geom, &hg);
            LAUE_CHECK_HIP(hipMemcpyAsync(sw[k].geom, &hg, sizeof(GeomF), hipMemcpyHostToDevice, s));
            LAUE_CHECK_HIP(hipMemcpyAsync(sw[k].mboff, a.model->block_off, (nb + 1) * sizeof(int64_t),
                                          hipMemcpyHostToDevice, s));
        }
        // heaviest items first across the batch
        std::stable_sort(rows.begin(), rows.end(),
                         [](const Item &a, const Item &b) { return (a.c1 - a.c0) > (b.c1 - b.c0); });
        std::stable_sort(cols.begin(), cols.end(),
                         [](const Item &a, const Item &b) { return (a.r1 - a.r0) > (b.r1 - b.r0); });
        n_rows = static_cast<int>(rows.size());
        n_cols = static_cast<int>(cols.size());
        // two-per-lane workgroups: adjacent items of one block and sample
        // (after the stable sort the items of a block stay contiguous)
        std::vector<int2> rows2, cols2;
        auto pair_up = [&](const std::vector<Item> &v, bool by_rows, std::vector<int2> &out, bool row_side) {
            for (size_t k = 0; k < v.size();) {
                const Item &a = v[k];
                bool pair = false;
                if (k + 1 < v.size()) {
                    const Item &b = v[k + 1];
                    pair = b.s == a.s && (by_rows ? (b.c0 == a.c0 && b.c1 == a.c1 && b.r0 == a.r1 && a.r1 > a.r0)
                                                  : (b.r0 == a.r0 && b.r1 == a.r1 && b.c0 == a.c1 && a.c1 > a.c0));
                }
                out.push_back(make_int2(static_cast<int>(k), pair ? static_cast<int>(k + 1) : -1));
                if (row_side) hd[a.s].n_row_wg2 += 1; else hd[a.s].n_col_wg2 += 1;
                k += pair ? 2 : 1;
            }
        };
        pair_up(rows, true, rows2, true);
        pair_up(cols, false, cols2, false);
        n_rows2 = static_cast<int>(rows2.size());
        n_cols2 = static_cast<int>(cols2.size());
        LAUE_CHECK_HIP(hipMemcpyAsync(bw.rows, rows.data(), rows.size() * sizeof(Item), hipMemcpyHostToDevice, s));
        LAUE_CHECK_HIP(hipMemcpyAsync(bw.cols, cols.data(), cols.size() * sizeof(Item), hipMemcpyHostToDevice, s));
        LAUE_CHECK_HIP(hipMemcpyAsync(bw.rows2, rows2.data(), rows2.size() * sizeof(int2), hipMemcpyHostToDevice, s));
        LAUE_CHECK_HIP(hipMemcpyAsync(bw.cols2, cols2.data(), cols2.size() * sizeof(int2), hipMemcpyHostToDevice, s));
        LAUE_CHECK_HIP(hipMemcpyAsync(bw.desc, hd.data(), n * sizeof(SampleDesc), hipMemcpyHostToDevice, s));
        LAUE_CHECK_HIP(hipMemcpyAsync(bw.mbase, mbase.data(), (n + 1) * sizeof(int64_t), hipMemcpyHostToDevice, s));
        LAUE_CHECK_HIP(hipMemcpyAsync(bw.gbase, gbase.data(), (n + 1) * sizeof(int64_t), hipMemcpyHostToDevice, s));
        LAUE_CHECK_HIP(hipStreamSynchronize(s));
        hctl.assign(n, SinkCtl{});
        return LAUE_OK;
    }

    int grain_prep() {
        if (gbase[n] == 0) return LAUE_OK;
        k_grain_prep_b<<<static_cast<unsigned>((gbase[n] + 255) / 256), 256, 0, s>>>(bw.desc, n, bw.gbase);
        LAUE_CHECK_HIP(hipGetLastError());
        return LAUE_OK;
    }

    int eval(int to_c, int with_outputs) {
        eval_on(s, to_c, with_outputs);
        LAUE_CHECK_HIP(hipGetLastError());
        return LAUE_OK;
    }

    void eval_on(hipStream_t st, int to_c, int with_outputs) {
        if (mbase[n] == 0) return;
        k_eval_b<<<static_cast<unsigned>((mbase[n] + 255) / 256), 256, 0, st>>>(bw.desc, n, bw.mbase, to_c,
                                                                                with_outputs);
    }

    // k_gn Gauss-Newton steps with the plan of (potentials, eps, colsE) fixed,
    // then the forward model at the new grains for the next E-step.
    // k_gn Gauss-Newton steps: statistics (dense or sparse) and the per-grain solve
    template <int MODE>
    void acc_pass(hipStream_t st, int cur_c) {
        if (mbase[n] == 0) return;
        if (rho > 0)
            k_mstep_acc_sparse<MODE><<<n_cols, 64, 0, st>>>(bw.cols, bw.desc, cur_c);
        else
            k_mstep_acc<MODE><<<n_cols, 64, 0, st>>>(bw.cols, bw.desc, cur_c);
    }

    void gn_steps(hipStream_t st, int k_gn) {
        const unsigned ng = static_cast<unsigned>(gbase[n]);
        if (mmethod == 1) {
            // k_gn sweeps: LauePosNewton (k_newton steps) on x, then LaueRotMM on R at the new x
            for (int sw_ = 0; sw_ < k_gn; ++sw_) {
                for (int it = 0; it < k_newton; ++it) {
                    const bool first = sw_ == 0 && it == 0;
                    if (!first) eval_on(st, 1, 0);
                    acc_pass<1>(st, first ? 0 : 1);
                    if (ng > 0) k_pos_solve<<<ng, 64, 0, st>>>(bw.desc, n, bw.gbase, it);
                }
                eval_on(st, 1, 0);
                acc_pass<2>(st, 1);
                if (ng > 0) k_rot_mm<<<ng, 64, 0, st>>>(bw.desc, n, bw.gbase);
            }
            return;
        }
        for (int k = 0; k < k_gn; ++k) {
            if (k > 0) eval_on(st, 1, 0);
            acc_pass<0>(st, k > 0 ? 1 : 0);
            if (ng > 0) k_mstep_solve<<<ng, 64, 0, st>>>(bw.desc, n, bw.gbase);
        }
    }

    // streamed M-step passes of k_gn steps (sweeps)
    int mstep_passes(int k_gn) const { return mmethod == 1 ? k_gn * (k_newton + 1) : k_gn; }

    void mstep_launches(hipStream_t st, int k_gn) {
        gn_steps(st, k_gn);
        eval_on(st, 0, 1);
    }

    // control blocks at temperature eps[k] from the potentials' bins.  gauge:
    // re-centre the potentials of every sample with the outlier row and column
    // to f0 = 0 first (k_gauge; the same plan)
    int init_ctl(const std::vector<double> &eps, bool gauge = false) {
        std::vector<CtlInit> v(n);
        int64_t longest = 0;
        for (int k = 0; k < n; ++k) {
            const SinkParams &sp = hd[k].sp;
            laue_potentials *pot = in[k].pot;
            double C = 0.0;
            if (gauge && !sp.unb && !sp.part && sp.t_b > 0 && std::isfinite(pot->f0) && pot->f0 != 0.0) {
                C = pot->f0;
                pot->f0 = 0.0;
                pot->g0 += C;
                longest = std::max(longest, std::max(in[k].obs->n, in[k].model->n));
            }
            v[k] = CtlInit{sp.t_b > 0 ? pot->f0 : -INFINITY, sp.t_a > 0 ? pot->g0 : -INFINITY, eps[k], C};
        }
        LAUE_CHECK_HIP(hipMemcpyAsync(bw.init, v.data(), n * sizeof(CtlInit), hipMemcpyHostToDevice, s));
        if (longest > 0)
            k_gauge<<<dim3(static_cast<unsigned>((longest + 255) / 256), n), 256, 0, s>>>(bw.desc, bw.init);
        k_ctl_init<<<(n + 63) / 64, 64, 0, s>>>(bw.desc, n, bw.init);
        LAUE_CHECK_HIP(hipGetLastError());
        // the host copy must outlive the asynchronous copy
        LAUE_CHECK_HIP(hipStreamSynchronize(s));
        return LAUE_OK;
    }

    int current_mode() const {
        if (launch_mode != 0) return launch_mode;
        if (chosen) return chosen;
        return t_direct < 0.0 ? 1 : 2;
    }

    // Sinkhorn of every sample from its potentials at temperature eps[k].
    // chunk: iterations between host polls (0: from the stage's history).
    int sinkhorn(const std::vector<double> &eps, int chunk, std::vector<laue_ot_stats> &st, int stage = -1) {
        int rc;
        // sparse: the neighbour sets of this E-step's columns
        if ((rc = build_neighbors())) return rc;
        if ((rc = init_ctl(eps, true))) return rc;
        // partial OT starts every solve from the Gibbs kernel (f = g = 0, H = 0)
        for (int k = 0; k < n; ++k) {
            if (!hd[k].sp.part) continue;
            const int64_t no = in[k].obs->n, nm = in[k].model->n;
            if (no > 0) k_fill_f<<<static_cast<unsigned>((no + 255) / 256), 256, 0, s>>>(in[k].pot->f, no, 0.0, 0);
            if (nm > 0) k_fill_f<<<static_cast<unsigned>((nm + 255) / 256), 256, 0, s>>>(in[k].pot->g, nm, 0.0, 0);
        }
        if (n_cols) {
            k_cs_init<<<n_cols, 64, 0, s>>>(bw.cols, bw.desc);
            k_cs_final<<<n, 256, 0, s>>>(bw.desc);
        }
        LAUE_CHECK_HIP(hipGetLastError());
        if (chunk <= 0) {
            chunk = 16;
            if (stage >= 0 && stage < static_cast<int>(stage_iters.size()) && stage_iters[stage] >= 0) {
                chunk = 4;
                while (chunk < stage_iters[stage] + 2 && chunk < 64) chunk <<= 1;
            }
        }
        int cap = 0;
        for (int k = 0; k < n; ++k) cap = std::max(cap, hd[k].sp.n_max);
        // tile shape of this Sinkhorn.  Tuning (the first Sinkhorn of a stage)
        // times row pass 2 in the one-per-lane shape and row pass 3 in the
        // two-per-lane shape, and the stage keeps the faster one.
        const int si = std::max(stage, 0);
        if (si >= static_cast<int>(stage_tile.size())) stage_tile.resize(si + 1, 0);
        int launched = 0;
        if (tile_mode == 0 && stage_tile[si] == 0 && rho == 0) {
            if (!tev[0])
                for (auto &e : tev) LAUE_CHECK_HIP(hipEventCreate(&e));
            // iteration 1 untimed (after a warm start it can take the slow
            // underflow path), then row pass 2 in shape 1 and row pass 3 in
            // shape 2 timed; if a sample converges within the three
            // iterations the later timing is not a full pass: keep shape 1
            LAUE_CHECK_HIP(hipEventRecord(tev[0], s));
            row_launch(s, 1);
            col_launch(s, 1);
            LAUE_CHECK_HIP(hipEventRecord(tev[1], s));
            row_launch(s, 1);
            LAUE_CHECK_HIP(hipEventRecord(tev[2], s));
            col_launch(s, 1);
            LAUE_CHECK_HIP(hipEventRecord(tev[3], s));
            row_launch(s, 2);
            LAUE_CHECK_HIP(hipEventRecord(tev[4], s));
            col_launch(s, 2);
            LAUE_CHECK_HIP(hipEventRecord(tev[5], s));
            LAUE_CHECK_HIP(hipGetLastError());
            LAUE_CHECK_HIP(hipMemcpyAsync(hctl.data(), bw.ctl, n * sizeof(SinkCtl), hipMemcpyDeviceToHost, s));
            LAUE_CHECK_HIP(hipEventSynchronize(tev[5]));
            LAUE_CHECK_HIP(hipStreamSynchronize(s));
            float t1 = 0.0f, t2 = 0.0f, tall = 0.0f;
            LAUE_CHECK_HIP(hipEventElapsedTime(&t1, tev[1], tev[2]));
            LAUE_CHECK_HIP(hipEventElapsedTime(&t2, tev[3], tev[4]));
            LAUE_CHECK_HIP(hipEventElapsedTime(&tall, tev[0], tev[5]));
            sink_ms += tall;
            bool any_done = false;
            for (int k = 0; k < n; ++k) any_done = any_done || hctl[k].done;
            stage_tile[si] = (!any_done && t2 < t1) ? 2 : 1;
            launched = 3;
        }
        const int R = rho > 0 ? 1 : (tile_mode ? tile_mode : std::max(stage_tile[si], 1));
        tiles_used.push_back(R);
        for (;;) {
            const int mode = current_mode();
            hipGraphExec_t gx = nullptr;
            if (mode == 2 && (rc = graph_for(chunk, R, &gx))) return rc;
            if ((rc = timer_start())) return rc;
            if (mode == 2) {
                LAUE_CHECK_HIP(hipGraphLaunch(gx, s));
            } else {
                for (int c = 0; c < chunk; ++c) pass_pair(s, R);
                LAUE_CHECK_HIP(hipGetLastError());
            }
            launched += chunk;
            double dt = 0.0;
            if ((rc = timer_stop(&sink_ms, &dt))) return rc;
            LAUE_CHECK_HIP(hipMemcpyAsync(hctl.data(), bw.ctl, n * sizeof(SinkCtl), hipMemcpyDeviceToHost, s));
            LAUE_CHECK_HIP(hipStreamSynchronize(s));
            ++polls;
            bool all = true, any = false;
            for (int k = 0; k < n; ++k) {
                all = all && hctl[k].done;
                any = any || hctl[k].done;
            }
            // tuning: a chunk in which no sample finished timed every pass at work
            if (launch_mode == 0 && !chosen && !any) {
                (mode == 2 ? t_graph : t_direct) = dt / chunk;
                if (t_direct >= 0.0 && t_graph >= 0.0) chosen = t_graph < t_direct ? 2 : 1;
            }
            if (all) break;
            if (launched > cap + 1) {
                set_error("internal: Sinkhorn did not stop at its cap");
                return LAUE_EDEVICE;
            }
        }
        if (stage >= 0) {
            if (stage >= static_cast<int>(stage_iters.size())) stage_iters.resize(stage + 1, -1);
            int mx = 0;
            for (int k = 0; k < n; ++k) mx = std::max(mx, hctl[k].final_state);
            stage_iters[stage] = mx;
        }
        st.assign(n, laue_ot_stats{});
        for (int k = 0; k < n; ++k) {
            const SinkCtl &h = hctl[k];
            const int fin = h.final_state;
            laue_potentials *pot = in[k].pot;
            if ((fin & 1) && in[k].obs->n > 0)
                LAUE_CHECK_HIP(hipMemcpyAsync(pot->f, sw[k].F1, in[k].obs->n * sizeof(float),
                                              hipMemcpyDeviceToDevice, s));
            // partial OT: fold the mass potential into f, so that Q = exp((f + g - c)/eps)
            if (hd[k].sp.part && in[k].obs->n > 0 && h.H != 0.0)
                k_fill_f<<<static_cast<unsigned>((in[k].obs->n + 255) / 256), 256, 0, s>>>(pot->f, in[k].obs->n, h.H,
                                                                                           1);
            pot->f0 = h.f0[fin & 1];
            pot->g0 = h.g0[fin & 1];
            st[k].n_iter = fin;
            st[k].converged = h.converged;
            st[k].err = h.err;
            const int64_t np = 2 * static_cast<int64_t>(fin) + 1;
            entries[k] += pass_work(k) * np;
            passes[k] += np;
            pass_entries[k] += pass_work(k) * np;
        }
        return LAUE_OK;
    }

    // k_gn Gauss-Newton steps with the plan of (potentials, eps, colsE) fixed
    // (launch mode 2: one captured graph), then the forward evaluation for
    // the next E-step (eval_next) or none (a lone M-step call).
    int mstep(int k_gn, bool eval_next) {
        int rc;
        if ((rc = timer_start())) return rc;
        if (eval_next && current_mode() == 2) {
            hipGraphExec_t gx = nullptr;
            if ((rc = mstep_graph(k_gn, &gx))) return rc;
            LAUE_CHECK_HIP(hipGraphLaunch(gx, s));
        } else {
            gn_steps(s, k_gn);
            if (eval_next) eval_on(s, 0, 1);
            LAUE_CHECK_HIP(hipGetLastError());
        }
        for (int j = 0; j < n; ++j) {
            entries[j] += pass_work(j) * mstep_passes(k_gn);
            m_entries[j] += pass_work(j) * mstep_passes(k_gn);
        }
        return timer_stop(&mstep_ms);
    }

    // the current plan of every sample (its temperature and final bin
    // potentials) into objin[0 .. n) (prev = 0) or objin[n .. 2n) (prev = 1)
    int set_objin(const std::vector<double> &eps, int prev) {
        std::vector<ObjIn> v(n);
        for (int k = 0; k < n; ++k) {
            const bool bins = !hd[k].sp.unb && !hd[k].sp.part;
            v[k] = ObjIn{eps[k], bins && hd[k].sp.t_b > 0 ? in[k].pot->f0 : -INFINITY,
                         bins && hd[k].sp.t_a > 0 ? in[k].pot->g0 : -INFINITY};
        }
        LAUE_CHECK_HIP(hipMemcpyAsync(bw.objin + (prev ? n : 0), v.data(), n * sizeof(ObjIn), hipMemcpyHostToDevice,
                                      s));
        LAUE_CHECK_HIP(hipStreamSynchronize(s));   // the host copy must outlive the copy
        return LAUE_OK;
    }

    // hard assignments (and Q_0j) of the current plan (set_objin first)
    int assign() {
        bool any = false, anyu = false;
        int64_t longest = 0;
        for (int k = 0; k < n; ++k) {
            any = any || (hd[k].jstar && in[k].obs->n > 0);
            if (hd[k].qunm && in[k].model->n > 0) {
                anyu = true;
                longest = std::max(longest, in[k].model->n);
            }
        }
        if (any) {
            if (rho > 0)
                k_assign_sparse<<<n_rows, 64, 0, s>>>(bw.rows, bw.desc);
            else
                k_assign<<<n_rows, 64, 0, s>>>(bw.rows, bw.desc);
            for (int k = 0; k < n; ++k)
                if (hd[k].jstar) entries[k] += pass_work(k);
        }
        if (anyu)
            k_assign_unm<<<dim3(static_cast<unsigned>((longest + 255) / 256), n), 256, 0, s>>>(bw.desc, bw.objin);
        LAUE_CHECK_HIP(hipGetLastError());
        return LAUE_OK;
    }

    // FP64 summaries of the current plan of every sample (set_objin first):
    // out[k] = (mass, <c,Q> matches, total cost, sum Q ln Q)
    int summaries(std::vector<std::array<double, 4>> &out) {
        if (n_rows) k_obj_rows<<<n_rows, 64, 0, s>>>(bw.rows, bw.desc, bw.objin);
        if (n_cols) k_obj_cols<<<n_cols, 64, 0, s>>>(bw.cols, bw.desc, bw.objin);
        k_obj_final<<<n, 64, 0, s>>>(bw.desc, bw.objin);
        LAUE_CHECK_HIP(hipGetLastError());
        out.assign(n, {0.0, 0.0, 0.0, 0.0});
        for (int k = 0; k < n; ++k) {
            const int64_t items = static_cast<int64_t>(hd[k].n_row_items) + hd[k].n_col_items;
            LAUE_CHECK_HIP(hipMemcpyAsync(out[k].data(), sw[k].obj + 4 * items, 4 * sizeof(double),
                                          hipMemcpyDeviceToHost, s));
        }
        LAUE_CHECK_HIP(hipStreamSynchronize(s));
        return LAUE_OK;
    }

    // the current plan becomes the previous one (columns, potentials, objin)
    int save_prev(const std::vector<double> &eps) {
        for (int k = 0; k < n; ++k) {
            if (in[k].model->n > 0) {
                LAUE_CHECK_HIP(hipMemcpyAsync(sw[k].colsP, sw[k].colsE, in[k].model->n * sizeof(Col8),
                                              hipMemcpyDeviceToDevice, s));
                LAUE_CHECK_HIP(hipMemcpyAsync(sw[k].Gp, in[k].pot->g, in[k].model->n * sizeof(float),
                                              hipMemcpyDeviceToDevice, s));
            }
            if (in[k].obs->n > 0)
                LAUE_CHECK_HIP(hipMemcpyAsync(sw[k].Fp, in[k].pot->f, in[k].obs->n * sizeof(float),
                                              hipMemcpyDeviceToDevice, s));
            if (rho > 0 && in[k].obs->n > 0)
                LAUE_CHECK_HIP(hipMemcpyAsync(sw[k].nbr_prev, sw[k].nbr, in[k].obs->n * rho * sizeof(int),
                                              hipMemcpyDeviceToDevice, s));
        }
        return set_objin(eps, 1);
    }

    // zeta = ||Q - Q_prev||_F of every sample (set_objin and save_prev first)
    int plan_change(std::vector<double> &zeta) {
        if (n_rows && rho > 0) k_dq_rows_sparse<<<n_rows, 64, 0, s>>>(bw.rows, bw.desc, bw.objin, n);
        else if (n_rows) k_dq_rows<<<n_rows, 64, 0, s>>>(bw.rows, bw.desc, bw.objin, n);
        if (n_cols) k_dq_cols<<<n_cols, 64, 0, s>>>(bw.cols, bw.desc, bw.objin, n);
        k_dq_final<<<n, 64, 0, s>>>(bw.desc, bw.objin, n);
        LAUE_CHECK_HIP(hipGetLastError());
        zeta.assign(n, 0.0);
        for (int k = 0; k < n; ++k) {
            const int64_t items = static_cast<int64_t>(hd[k].n_row_items) + hd[k].n_col_items;
            LAUE_CHECK_HIP(hipMemcpyAsync(&zeta[k], sw[k].obj + 4 * items, sizeof(double), hipMemcpyDeviceToHost,
                                          s));
        }
        LAUE_CHECK_HIP(hipStreamSynchronize(s));
        for (int k = 0; k < n; ++k) entries[k] += 2 * pass_work(k);
        return LAUE_OK;
    }
};

// Temperatures of an EM run: the stage schedule (n_stages x iters_per_stage,
// geometric from eps_start to eps_end) or, with eps_cool in (0, 1), the
// cooling of Alg. LaueOT (Sec. 5.1): eps_start, then times eps_cool while the
// last one is above eps_end (FP64 products in this order).
static std::vector<double> em_temperatures(const laue_em_params &p) {
    std::vector<double> t;
    if (p.eps_cool > 0.0) {
        t.push_back(p.eps_start);
        while (t.back() > p.eps_end) t.push_back(t.back() * p.eps_cool);
        return t;
    }
    const int S = p.n_stages;
    for (int st = 0; st < S; ++st) {
        const double e = S == 1 ? p.eps_start
                                : p.eps_start * std::pow(p.eps_end / p.eps_start, static_cast<double>(st) / (S - 1));
        for (int it = 0; it < p.iters_per_stage; ++it) t.push_back(e);
    }
    return t;
}

int em_n_temperatures(const laue_em_params &p) { return static_cast<int>(em_temperatures(p).size()); }

static int run_em(BatchEngine &e, const std::vector<const laue_em_params *> &par, std::vector<laue_em_stats> &stats) {
    int rc;
    const int n = e.n;
    if ((rc = e.grain_prep())) return rc;
    stats.assign(n, laue_em_stats{});
    e.launch_mode = par[0]->launch;
    e.tile_mode = par[0]->tile;
    std::vector<std::vector<double>> temps(n);
    for (int k = 0; k < n; ++k) temps[k] = em_temperatures(*par[k]);
    const int L = static_cast<int>(temps[0].size());
    for (int k = 1; k < n; ++k)
        LAUE_REQUIRE(static_cast<int>(temps[k].size()) == L, LAUE_EINVAL,
                     "samples of a batch need the same number of EM temperatures");
    const bool cooling = par[0]->eps_cool > 0.0;
    const int n_final = cooling ? par[0]->final_iters : 0;
    const bool zeta_on = cooling && n == 1;
    const bool zeta_stop = zeta_on && par[0]->zeta_tol > 0.0;
    const int total = L + n_final;
    // the stage of a temperature (chunk sizing and tile tuning): the stage
    // index, or one stage per eight cooling steps
    const int ips = std::max(par[0]->iters_per_stage, 1);
    std::vector<double> eps(n), zeta;
    std::vector<laue_ot_stats> os;
    for (int k = 0; k < n; ++k) {
        stats[k].zeta = NAN;
        stats[k].objective = laue_objective{NAN, NAN, NAN, NAN, NAN};
    }
    bool have_prev = false;
    for (int it = 0; it < total; ++it) {
        for (int k = 0; k < n; ++k) eps[k] = temps[k][std::min(it, L - 1)];
        const int stage = cooling ? std::min(it, L) / 8 : it / ips;
        if (it == 0 && (rc = e.eval(0, 1))) return rc;    // later: after each M-step
        if ((rc = e.sinkhorn(eps, par[0]->ot.chunk, os, stage))) return rc;
        for (int k = 0; k < n; ++k) {
            stats[k].sinkhorn_iters += os[k].n_iter;
            stats[k].not_converged += os[k].converged ? 0 : 1;
            stats[k].last_err = os[k].err;
            stats[k].n_em_iter += 1;
            if (it >= L) stats[k].final_iters_run += 1;
        }
        bool last = it == total - 1;
        // the plan change from the previous EM iteration (Alg. LaueOT's stop)
        if (zeta_on && it >= L - 1) {
            if ((rc = e.set_objin(eps, 0))) return rc;
            if (have_prev) {
                if ((rc = e.plan_change(zeta))) return rc;
                stats[0].zeta = zeta[0];
                if (zeta_stop && zeta[0] <= par[0]->zeta_tol) last = true;
            }
        }
        if (zeta_on && it >= L - 2 && !last) {
            if ((rc = e.set_objin(eps, 0)) || (rc = e.save_prev(eps))) return rc;
            have_prev = true;
        }
        // Alg. LaueOT's outputs: the last E-step's plan (assignments, likelihood)
        if (last) {
            if ((rc = e.set_objin(eps, 0)) || (rc = e.assign())) return rc;
            bool want = false;
            for (int k = 0; k < n; ++k) want = want || par[k]->sigma_mm > 0.0;
            if (want) {
                std::vector<std::array<double, 4>> t;
                if ((rc = e.summaries(t))) return rc;
                for (int k = 0; k < n; ++k) {
                    if (!(par[k]->sigma_mm > 0.0)) continue;
                    laue_objective &o = stats[k].objective;
                    o.mass = t[k][0];
                    o.cost_inlier = t[k][1];
                    o.cost_total = t[k][2];
                    o.entropy = -t[k][3];
                    const bool bins = !e.hd[k].sp.unb && !e.hd[k].sp.part;
                    const double sg = par[k]->sigma_mm, s2 = 2.0 * sg * sg;
                    const double kap = (par[k]->ot.distance / sg) * (par[k]->ot.distance / sg);
                    o.sem_objective = bins ? kap * t[k][0] - t[k][2] / s2 + eps[k] / s2 * (-t[k][3]) : NAN;
                }
            }
        }
        // all samples share k_gn (checked by the caller); the M-step ends
        // with the forward evaluation at the new grains
        if ((rc = e.mstep(par[0]->gn.k_gn, true))) return rc;
        if (last) break;
    }
    for (int k = 0; k < n; ++k) {
        stats[k].cost_entries = e.entries[k];
        stats[k].sinkhorn_ms = e.sink_ms;
        stats[k].sinkhorn_passes = e.passes[k];
        stats[k].sinkhorn_entries = e.pass_entries[k];
        stats[k].mstep_ms = e.mstep_ms;
        stats[k].mstep_entries = e.m_entries[k];
        stats[k].launch_used = e.current_mode();
        stats[k].polls = e.polls;
        int t2 = 0;
        for (int t : e.tiles_used) t2 += t == 2;
        stats[k].tile2_solves = t2;
    }
    LAUE_CHECK_HIP(hipStreamSynchronize(e.s));
    return LAUE_OK;
}

}  // namespace laue

using namespace laue;

static std::vector<SampleDims> dims_of(int n, const laue_geometry *geoms, const int64_t *n_obs, const int64_t *n_model,
                                       const int32_t *n_grains) {
    std::vector<SampleDims> d(n);
    for (int k = 0; k < n; ++k) d[k] = SampleDims{geoms + k, n_obs[k], n_model[k], n_grains ? n_grains[k] : 0, 0};
    return d;
}

extern "C" size_t laue_sinkhorn_workspace_size(const laue_geometry *geom, int64_t n_obs,
                                               int64_t n_model, int32_t n_grains) {
    if (!geom || validate_geometry(geom) != LAUE_OK || n_obs < 0 || n_model < 0 || n_grains < 0)
        return 0;
    Carver cv(nullptr);
    BatchWs bw;
    std::vector<SampleWs> sw;
    return carve_all(cv, bw, sw, dims_of(1, geom, &n_obs, &n_model, &n_grains));
}

extern "C" size_t laue_sparse_workspace_size(int32_t n, const laue_geometry *geoms, const int64_t *n_obs,
                                             const int64_t *n_model, const int32_t *n_grains, int32_t rho) {
    if (n < 1 || !geoms || !n_obs || !n_model || (rho != 0 && rho != 8 && rho != 16 && rho != 32)) return 0;
    for (int k = 0; k < n; ++k)
        if (validate_geometry(geoms + k) != LAUE_OK || n_obs[k] < 0 || n_model[k] < 0 ||
            (n_grains && n_grains[k] < 0))
            return 0;
    std::vector<SampleDims> d = dims_of(n, geoms, n_obs, n_model, n_grains);
    for (auto &x : d) x.rho = rho;
    Carver cv(nullptr);
    BatchWs bw;
    std::vector<SampleWs> sw;
    return carve_all(cv, bw, sw, d);
}

extern "C" size_t laue_em_batched_workspace_size(int32_t n, const laue_geometry *geoms, const int64_t *n_obs,
                                                 const int64_t *n_model, const int32_t *n_grains) {
    if (n < 1 || !geoms || !n_obs || !n_model || !n_grains) return 0;
    for (int k = 0; k < n; ++k)
        if (validate_geometry(geoms + k) != LAUE_OK || n_obs[k] < 0 || n_model[k] < 0 || n_grains[k] < 0) return 0;
    Carver cv(nullptr);
    BatchWs bw;
    std::vector<SampleWs> sw;
    return carve_all(cv, bw, sw, dims_of(n, geoms, n_obs, n_model, n_grains));
}

// ---------------------------------------------------------------- objectives

extern "C" int laue_sinkhorn(const laue_geometry *geom, const laue_obs_spots *obs,
                             const laue_model_spots *model, const laue_ot_params *par,
                             laue_potentials *pot, laue_ot_stats *stats, void *ws, size_t ws_bytes,
                             void *stream) {
    clear_error();
    int rc;
    if ((rc = validate_ot(par, true))) return rc;
    LAUE_REQUIRE(pot && stats, LAUE_EINVAL, "potentials or stats is NULL");
    LAUE_REQUIRE(bins_ok(par, pot), LAUE_EINVAL, "bin potentials must be finite");
    BatchEngine e;
    laue_model_spots *m = const_cast<laue_model_spots *>(model);
    if ((rc = e.setup({SampleIn{geom, nullptr, obs, m, par, nullptr, pot, 0.0, nullptr, nullptr}}, ws, ws_bytes,
                      stream, true)))
        return rc;
    if ((rc = launch_pack(model, e.sw[0].colsE, e.s))) return rc;
    std::vector<laue_ot_stats> os;
    if ((rc = e.sinkhorn({par->eps}, par->chunk, os))) return rc;
    *stats = os[0];
    LAUE_CHECK_HIP(hipStreamSynchronize(e.s));
    return stats->converged ? LAUE_OK : LAUE_ENOCONV;
}

// ---------------------------------------------------------------- allocation-free Sinkhorn

// Scratch of laue_sinkhorn_noalloc: a file-scope device array that each GPU
// holds from the library's first use until the process ends.  Host code never
// passes the array's name to a kernel (on the host it is only a stand-in for
// the symbol): the device address comes from hipGetSymbolAddress, once per
// device with that device current, and is kept per device.
namespace {
constexpr size_t kNoAllocScratchBytes = size_t(64) << 20;
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

int scratch_of_current_device(void **out) {
    int dev = -1;
    LAUE_CHECK_HIP(hipGetDevice(&dev));
    LAUE_REQUIRE(dev >= 0 && dev < kMaxDevices, LAUE_EDEVICE, "device index out of range");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        LAUE_CHECK_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        LAUE_REQUIRE(p != nullptr && (reinterpret_cast<uintptr_t>(p) & 255) == 0, LAUE_EDEVICE,
                     "scratch symbol has no aligned device address");
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return LAUE_OK;
}
}  // namespace

extern "C" size_t laue_sinkhorn_noalloc_capacity(void) { return kNoAllocScratchBytes; }

extern "C" int laue_sinkhorn_noalloc(const laue_geometry *geom, const laue_obs_spots *obs,
                                     const laue_model_spots *model, const laue_ot_params *par,
                                     laue_potentials *pot, laue_ot_stats *stats, void *stream) {
    clear_error();
    int rc;
    if ((rc = validate_ot(par, true))) return rc;
    LAUE_REQUIRE(pot && stats && obs && model, LAUE_EINVAL, "NULL argument");
    LAUE_REQUIRE(bins_ok(par, pot), LAUE_EINVAL, "bin potentials must be finite");
    if ((rc = validate_geometry(geom))) return rc;
    const size_t need =
        par->rho > 0
            ? laue_sparse_workspace_size(1, geom, &obs->n, &model->n, std::array<int32_t, 1>{0}.data(), par->rho)
            : laue_sinkhorn_workspace_size(geom, obs->n, model->n, 0);
    LAUE_REQUIRE(need > 0, LAUE_EINVAL, "bad problem sizes");
    LAUE_REQUIRE(need <= kNoAllocScratchBytes, LAUE_ECAPACITY,
                 "the problem needs " + std::to_string(need) + " bytes of scratch; laue_sinkhorn_noalloc holds " +
                     std::to_string(kNoAllocScratchBytes) + " (use laue_sinkhorn with a workspace)");
    void *ws = nullptr;
    if ((rc = scratch_of_current_device(&ws))) return rc;
    BatchEngine e;
    e.timing = false;
    laue_model_spots *m = const_cast<laue_model_spots *>(model);
    if ((rc = e.setup({SampleIn{geom, nullptr, obs, m, par, nullptr, pot, 0.0, nullptr, nullptr}}, ws,
                      kNoAllocScratchBytes, stream, true)))
        return rc;
    if ((rc = launch_pack(model, e.sw[0].colsE, e.s))) return rc;
    std::vector<laue_ot_stats> os;
    if ((rc = e.sinkhorn({par->eps}, par->chunk, os))) return rc;
    *stats = os[0];
    LAUE_CHECK_HIP(hipStreamSynchronize(e.s));
    return stats->converged ? LAUE_OK : LAUE_ENOCONV;
}

extern "C" int laue_objectives(const laue_geometry *geom, const laue_obs_spots *obs,
                               const laue_model_spots *model, const laue_ot_params *par,
                               const laue_potentials *pot, double sigma_mm, laue_objective *out, void *ws,
                               size_t ws_bytes, void *stream) {
    clear_error();
    int rc;
    if ((rc = validate_ot(par, true))) return rc;
    LAUE_REQUIRE(pot && out, LAUE_EINVAL, "potentials or output is NULL");
    LAUE_REQUIRE(std::isfinite(sigma_mm) && sigma_mm > 0, LAUE_EINVAL, "sigma_mm must be > 0");
    LAUE_REQUIRE(bins_ok(par, pot), LAUE_EINVAL, "bin potentials must be finite");
    BatchEngine e;
    laue_potentials p = *pot;           // read only
    laue_model_spots *m = const_cast<laue_model_spots *>(model);
    if ((rc = e.setup({SampleIn{geom, nullptr, obs, m, par, nullptr, &p, 0.0, nullptr, nullptr}}, ws, ws_bytes,
                      stream, true)))
        return rc;
    if ((rc = launch_pack(model, e.sw[0].colsE, e.s))) return rc;
    if ((rc = e.build_neighbors())) return rc;
    std::vector<std::array<double, 4>> t;
    if ((rc = e.set_objin({par->eps}, 0)) || (rc = e.summaries(t))) return rc;
    const bool bins = par->outlier_model == 0;
    out->mass = t[0][0];
    out->cost_inlier = t[0][1];
    out->cost_total = t[0][2];
    out->entropy = -t[0][3];
    const double s2 = 2.0 * sigma_mm * sigma_mm;
    const double kappa = (par->distance / sigma_mm) * (par->distance / sigma_mm);
    out->sem_objective = bins ? kappa * t[0][0] - t[0][2] / s2 + par->eps / s2 * (-t[0][3]) : NAN;
    return LAUE_OK;
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


extern "C" int laue_sparse_neighbors(const laue_geometry *geom, const laue_obs_spots *obs,
                                     const laue_model_spots *model, const laue_ot_params *par, int32_t *nbr,
                                     float *cost, int64_t *n_pairs, void *ws, size_t ws_bytes, void *stream) {
    clear_error();
    int rc;
    if ((rc = validate_ot(par, false))) return rc;
    LAUE_REQUIRE(par->rho > 0, LAUE_EINVAL, "rho must be 8, 16 or 32");
    LAUE_REQUIRE(obs && (obs->n == 0 || (nbr && cost)), LAUE_EINVAL, "output arrays are NULL");
    BatchEngine e;
    laue_model_spots *m = const_cast<laue_model_spots *>(model);
    laue_potentials pot{nullptr, nullptr, 0.0, 0.0};
    // the potentials are not read; give the setup checks something to hold
    float dummy = 0.0f;
    pot.f = &dummy;
    pot.g = &dummy;
    if ((rc = e.setup({SampleIn{geom, nullptr, obs, m, par, nullptr, &pot, 0.0, nullptr, nullptr}}, ws, ws_bytes,
                      stream, true)))
        return rc;
    if ((rc = launch_pack(model, e.sw[0].colsE, e.s))) return rc;
    if ((rc = e.build_neighbors())) return rc;
    const int64_t ne = obs->n * static_cast<int64_t>(par->rho);
    if (ne > 0) {
        k_knn_out<<<static_cast<unsigned>((ne + 255) / 256), 256, 0, e.s>>>(
            e.sw[0].nbr, e.sw[0].ncp, obs->n, par->rho, static_cast<float>(2.0 * par->distance * par->distance), nbr,
            cost);
        LAUE_CHECK_HIP(hipGetLastError());
    }
    if (n_pairs) *n_pairs = e.sparse_entries[0];
    LAUE_CHECK_HIP(hipStreamSynchronize(e.s));
    return LAUE_OK;
}

// cost of each detected spot's farthest kept neighbour (mm^2), -1 when it has none
__global__ void k_far_cost(const SampleDesc *__restrict__ descs, float *__restrict__ far) {
    const SampleDesc &D = descs[0];
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= D.n_obs) return;
    float c = -1.0f;
    for (int q = D.rho - 1; q >= 0; --q)
        if (D.nbr[q * D.n_obs + i] >= 0) {
            c = D.ncp[q * D.n_obs + i] * D.sp.twoD2;
            break;
        }
    far[i] = c;
}

extern "C" int laue_eps_init(const laue_geometry *geom, const laue_obs_spots *obs, const laue_model_spots *model,
                             const laue_ot_params *par, double *eps_init, void *ws, size_t ws_bytes, void *stream) {
    clear_error();
    int rc;
    if ((rc = validate_ot(par, false))) return rc;
    LAUE_REQUIRE(par->rho > 0, LAUE_EINVAL, "rho must be 8, 16 or 32");
    LAUE_REQUIRE(eps_init != nullptr && obs != nullptr, LAUE_EINVAL, "NULL argument");
    BatchEngine e;
    laue_model_spots *m = const_cast<laue_model_spots *>(model);
    laue_potentials pot{nullptr, nullptr, 0.0, 0.0};
    float dummy = 0.0f;     // the potentials are not read
    pot.f = &dummy;
    pot.g = &dummy;
    if ((rc = e.setup({SampleIn{geom, nullptr, obs, m, par, nullptr, &pot, 0.0, nullptr, nullptr}}, ws, ws_bytes,
                      stream, true)))
        return rc;
    if ((rc = launch_pack(model, e.sw[0].colsE, e.s))) return rc;
    if ((rc = e.build_neighbors())) return rc;
    *eps_init = 1.0;
    if (obs->n == 0) return LAUE_OK;
    float *far = e.sw[0].Fp;        // [n_obs] of the workspace
    k_far_cost<<<static_cast<unsigned>((obs->n + 255) / 256), 256, 0, e.s>>>(e.bw.desc, far);
    LAUE_CHECK_HIP(hipGetLastError());
    std::vector<float> h(obs->n);
    LAUE_CHECK_HIP(hipMemcpyAsync(h.data(), far, obs->n * sizeof(float), hipMemcpyDeviceToHost, e.s));
    LAUE_CHECK_HIP(hipStreamSynchronize(e.s));
    std::vector<double> v;
    v.reserve(h.size());
    for (float c : h)
        if (c >= 0.0f) v.push_back(static_cast<double>(c));
    if (v.empty()) return LAUE_OK;
    const size_t mid = v.size() / 2;
    std::nth_element(v.begin(), v.begin() + mid, v.end());
    double med = v[mid];
    if (v.size() % 2 == 0) med = 0.5 * (med + *std::max_element(v.begin(), v.begin() + mid));
    *eps_init = med / std::log(100.0);
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
    if ((rc = validate_gn(gn))) return rc;
    LAUE_REQUIRE(pot && obs && (obs->n == 0 || pot->f) && (model == nullptr || model->n == 0 || pot->g),
                 LAUE_EINVAL, "potentials are NULL");
    LAUE_REQUIRE(bins_ok(par, pot), LAUE_EINVAL, "bin potentials must be finite");
    BatchEngine e;
    laue_potentials p = *pot;           // read only
    if ((rc = e.setup({SampleIn{geom, planes, obs, model, par, grains, &p, gn->mu_rel, nullptr, step_norm, gn}}, ws,
                      ws_bytes, stream, true)))
        return rc;
    if ((rc = launch_pack(model, e.sw[0].colsE, e.s))) return rc;
    // sparse: the same neighbour sets as the E-step on these columns
    if ((rc = e.build_neighbors())) return rc;
    if ((rc = e.grain_prep()) || (rc = e.init_ctl({par->eps})) || (rc = e.mstep(gn->k_gn, false))) return rc;
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
    if ((rc = validate_em_params(par)) || (rc = validate_planes(planes)) || (rc = validate_grains(grains)))
        return rc;
    LAUE_REQUIRE(bins_ok(&par->ot, pot), LAUE_EINVAL, "bin potentials must be finite");
    BatchEngine e;
    if ((rc = e.setup({SampleIn{geom, planes, obs, model, &par->ot, grains, pot, par->gn.mu_rel, assign, nullptr,
                                &par->gn}},
                      ws, ws_bytes, stream, false)))
        return rc;
    std::vector<laue_em_stats> st;
    if ((rc = run_em(e, {par}, st))) return rc;
    *stats = st[0];
    return stats->not_converged ? LAUE_ENOCONV : LAUE_OK;
}

extern "C" int laue_em_batched(int32_t n, const laue_geometry *geoms, const laue_planes *planes,
                               const laue_obs_spots *obs, laue_model_spots *models, const laue_em_params *pars,
                               laue_grains *grains, laue_potentials *pots, laue_assignments *assigns,
                               laue_em_stats *stats, void *ws, size_t ws_bytes, void *stream) {
    clear_error();
    int rc;
    LAUE_REQUIRE(n >= 1 && geoms && planes && obs && models && pars && grains && pots && stats, LAUE_EINVAL,
                 "NULL argument");
    std::vector<SampleIn> in(n);
    std::vector<const laue_em_params *> par(n);
    for (int k = 0; k < n; ++k) {
        if ((rc = validate_em_params(pars + k)) || (rc = validate_planes(planes + k)) ||
            (rc = validate_grains(grains + k)))
            return rc;
        LAUE_REQUIRE(pars[k].n_stages == pars[0].n_stages && pars[k].iters_per_stage == pars[0].iters_per_stage &&
                         pars[k].gn.k_gn == pars[0].gn.k_gn,
                     LAUE_EINVAL, "samples of a batch share n_stages, iters_per_stage and k_gn");
        LAUE_REQUIRE(pars[k].launch == pars[0].launch && pars[k].ot.chunk == pars[0].ot.chunk &&
                         pars[k].tile == pars[0].tile,
                     LAUE_EINVAL, "samples of a batch share launch, tile and ot.chunk");
        LAUE_REQUIRE(pars[k].eps_cool == pars[0].eps_cool && pars[k].final_iters == pars[0].final_iters,
                     LAUE_EINVAL, "samples of a batch share eps_cool and final_iters");
        LAUE_REQUIRE(!(pars[k].eps_cool > 0.0 && pars[k].zeta_tol > 0.0), LAUE_EINVAL,
                     "the plan-change stop runs in laue_em only (one sample)");
        LAUE_REQUIRE(bins_ok(&pars[k].ot, pots + k), LAUE_EINVAL, "bin potentials must be finite");
        in[k] = SampleIn{geoms + k, planes + k, obs + k, models + k, &pars[k].ot, grains + k, pots + k,
                         pars[k].gn.mu_rel, assigns ? assigns + k : nullptr, nullptr, &pars[k].gn};
        par[k] = pars + k;
    }
    BatchEngine e;
    if ((rc = e.setup(in, ws, ws_bytes, stream, false))) return rc;
    std::vector<laue_em_stats> st;
    if ((rc = run_em(e, par, st))) return rc;
    int nc = 0;
    for (int k = 0; k < n; ++k) {
        stats[k] = st[k];
        nc += st[k].not_converged;
    }
    return nc ? LAUE_ENOCONV : LAUE_OK;
}
