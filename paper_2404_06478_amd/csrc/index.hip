// Prototype scoring (paper Sec. 6, App. D-E; Algs. SingleLaueOT and
// LaueSpotGreedy): spot-pair candidate orientations, single-grain refinement
// with a row-softmax E-step, the unmatched (3 sigma) filter, the sparse SPOT
// grain-to-spot matrix and greedy prototype selection.
//
// Candidate work is laid out by (block, candidate): one wave per pair, its
// lanes over the block's detected spots (64 at a time) and the candidate's few
// model spots of that block streamed as wave-uniform (scalar) loads.  The
// softmax normaliser of a detected spot is then a plain per-lane sum, and the
// M-step statistics of model spot j are wave-reduced and kept by lane j.
#include <algorithm>
#include <cmath>

#include <hipcub/hipcub.hpp>

#include "common.h"

namespace laue {

constexpr int kMaxReps = 128;

// ---------------------------------------------------------------- candidates

// Sample-frame plane normal n and sin(theta) of a detected spot read as a
// reflection of a grain at the sample centre: rhat = p/|p|, u = (e - rhat)/|e - rhat|,
// sin(theta) = |e - rhat|/2 (Eqs. ray_r, bragg), n = Gamma_t^T u.  FP64.
__device__ inline void spot_normal(const laue_geometry &G, int b, float p1, float p2, double *n,
                                   double &sth, double *plab) {
    const int t = b / G.n_det, d = b - t * G.n_det;
    const laue_detector &D = G.det[d];
    double nrm = 0.0;
    for (int k = 0; k < 3; ++k) {
        plab[k] = D.center[k] + static_cast<double>(p1) * D.axis1[k] + static_cast<double>(p2) * D.axis2[k];
        nrm += plab[k] * plab[k];
    }
    nrm = sqrt(nrm);
    double dv[3] = {1.0 - plab[0] / nrm, -plab[1] / nrm, -plab[2] / nrm};
    const double nd = sqrt(dv[0] * dv[0] + dv[1] * dv[1] + dv[2] * dv[2]);
    const double inv = nd > 0.0 ? 1.0 / nd : 0.0;
    const double u[3] = {dv[0] * inv, dv[1] * inv, dv[2] * inv};
    const double om = G.omega0 + G.domega * t, c = cos(om), s = sin(om);
    n[0] = c * u[0] + s * u[1];
    n[1] = -s * u[0] + c * u[1];
    n[2] = u[2];
    sth = 0.5 * nd;
}

// Wahba's problem (App. A) for three vector pairs: R minimising
// sum_k ||a_k - R b_k||^2 (rows of a and b), by wahba_quat_B.
__device__ inline void wahba_quat(const double a[3][3], const double b[3][3], double *q) {
    double B[3][3] = {};
    for (int k = 0; k < 3; ++k)
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) B[i][j] += a[k][i] * b[k][j];
    wahba_quat_B(B, q);
}

__device__ __forceinline__ void cross3(const double *a, const double *b, double *c) {
    c[0] = a[1] * b[2] - a[2] * b[1];
    c[1] = a[2] * b[0] - a[0] * b[2];
    c[2] = a[0] * b[1] - a[1] * b[0];
}

struct PairTab {
    int n_rep;
    int M;
    int rep[kMaxReps];
};

// One thread per pair k.  pass 0 counts hypotheses, pass 1 writes them at
// offs[k] (only below capacity).
__global__ void k_pairs(int pass, const laue_geometry G, const float *__restrict__ P1,
                        const float *__restrict__ P2, const int64_t *__restrict__ ooff,
                        const float *__restrict__ W, const float *__restrict__ Dsp,
                        const PairTab *__restrict__ tab, const double *__restrict__ angw,
                        const float *__restrict__ nrat, int64_t n_pairs, uint32_t k0, uint32_t k1,
                        double delta, double l_side, int *__restrict__ counts,
                        const int64_t *__restrict__ offs, int64_t cap, double *__restrict__ oq,
                        int *__restrict__ opair, int *__restrict__ oma, int *__restrict__ omb,
                        int *__restrict__ oa, int *__restrict__ ob, float *__restrict__ ofeat,
                        const int *__restrict__ pair_a, const int *__restrict__ pair_b) {
    const int64_t k = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (k >= n_pairs) return;
    const int nbk = G.n_rot * G.n_det;
    int t = 0;
    int64_t a = -1, b = -1;
    if (pair_a) {
        // explicit pair: both spots must lie in one rotation
        const int64_t pa = pair_a[k], pb = pair_b[k];
        if (pa >= 0 && pb >= 0 && pa < ooff[nbk] && pb < ooff[nbk]) {
            int lo = 0, hi = nbk;
            while (hi - lo > 1) {
                const int mid = (lo + hi) / 2;
                if (ooff[mid] <= pa) lo = mid; else hi = mid;
            }
            t = lo / G.n_det;
            if (pb >= ooff[t * G.n_det] && pb < ooff[(t + 1) * G.n_det]) {
                a = pa;
                b = pb;
            }
        }
    } else {
        uint32_t c[4] = {static_cast<uint32_t>(k), 0u, 0u, 5u};
        philox(c, k0, k1);
        t = static_cast<int>(c[0] % static_cast<uint32_t>(G.n_rot));
        const int64_t lo = ooff[t * G.n_det], hi = ooff[(t + 1) * G.n_det];
        const uint32_t cnt = static_cast<uint32_t>(hi - lo);
        if (cnt > 0) {
            a = lo + c[1] % cnt;
            b = lo + c[2] % cnt;
        }
    }
    int found = 0;
    int64_t base = pass ? offs[k] : 0;
    if (a >= 0) {
        if (a != b) {
            int ba = t * G.n_det, bb = t * G.n_det;
            while (ba + 1 < (t + 1) * G.n_det && ooff[ba + 1] <= a) ++ba;
            while (bb + 1 < (t + 1) * G.n_det && ooff[bb + 1] <= b) ++bb;
            double na[3], nb[3], pa[3], pb[3], sa, sb;
            spot_normal(G, ba, P1[a], P2[a], na, sa, pa);
            spot_normal(G, bb, P1[b], P2[b], nb, sb, pb);
            double cab = na[0] * nb[0] + na[1] * nb[1] + na[2] * nb[2];
            cab = fmin(1.0, fmax(-1.0, cab));
            const double ang_n = acos(cab);
            const int M = tab->M;
            const double lmin = G.lambda_min, lmax = G.lambda_max;
            for (int r = 0; r < tab->n_rep; ++r) {
                const int ma = tab->rep[r];
                const double la = 2.0 * static_cast<double>(Dsp[ma]) * sa;
                if (!(la >= lmin && la <= lmax)) continue;
                for (int mb = 0; mb < M; ++mb) {
                    const double aw = angw[static_cast<int64_t>(r) * M + mb];
                    if (!(aw >= 0.0)) continue;          // parallel planes are marked NaN
                    if (!(fabs(aw - ang_n) <= delta)) continue;
                    const double lb = 2.0 * static_cast<double>(Dsp[mb]) * sb;
                    if (!(lb >= lmin && lb <= lmax)) continue;
                    if (pass) {
                        const int64_t pos = base + found;
                        if (pos < cap) {
                            double wa[3] = {W[3 * ma], W[3 * ma + 1], W[3 * ma + 2]};
                            double wb[3] = {W[3 * mb], W[3 * mb + 1], W[3 * mb + 2]};
                            double cn[3], cw[3];
                            cross3(na, nb, cn);
                            cross3(wa, wb, cw);
                            const double ln = sqrt(cn[0] * cn[0] + cn[1] * cn[1] + cn[2] * cn[2]);
                            const double lw = sqrt(cw[0] * cw[0] + cw[1] * cw[1] + cw[2] * cw[2]);
                            double A[3][3], Bm[3][3];
                            for (int i = 0; i < 3; ++i) {
                                A[0][i] = na[i];
                                A[1][i] = nb[i];
                                A[2][i] = ln > 0 ? cn[i] / ln : 0.0;
                                Bm[0][i] = wa[i];
                                Bm[1][i] = wb[i];
                                Bm[2][i] = lw > 0 ? cw[i] / lw : 0.0;
                            }
                            double q[4];
                            wahba_quat(A, Bm, q);
                            for (int i = 0; i < 4; ++i) oq[4 * pos + i] = q[i];
                            if (opair) opair[pos] = static_cast<int>(k);
                            if (oma) oma[pos] = ma;
                            if (omb) omb[pos] = mb;
                            if (oa) oa[pos] = static_cast<int>(a);
                            if (ob) ob[pos] = static_cast<int>(b);
                            if (ofeat) {
                                float *f = ofeat + 16 * pos;
                                const double dw = wa[0] * wb[0] + wa[1] * wb[1] + wa[2] * wb[2];
                                double dp = 0.0;
                                for (int i = 0; i < 3; ++i) dp += (pa[i] - pb[i]) * (pa[i] - pb[i]);
                                f[0] = static_cast<float>(cab);
                                f[1] = static_cast<float>(dw);
                                f[2] = static_cast<float>(fabs(aw - ang_n) / delta);
                                f[3] = static_cast<float>(sa);
                                f[4] = static_cast<float>(sb);
                                f[5] = static_cast<float>((la - lmin) / (lmax - lmin));
                                f[6] = static_cast<float>((lb - lmin) / (lmax - lmin));
                                f[7] = nrat[ma];
                                f[8] = nrat[mb];
                                f[9] = static_cast<float>(sqrt(dp) / (2.0 * l_side));
                                f[10] = static_cast<float>(sqrt(static_cast<double>(P1[a]) * P1[a] +
                                                                static_cast<double>(P2[a]) * P2[a]) / l_side);
                                f[11] = static_cast<float>(sqrt(static_cast<double>(P1[b]) * P1[b] +
                                                                static_cast<double>(P2[b]) * P2[b]) / l_side);
                                f[12] = static_cast<float>(ba - t * G.n_det);
                                f[13] = static_cast<float>(bb - t * G.n_det);
                                f[14] = 0.0f;
                                f[15] = 0.0f;
                            }
                        }
                    }
                    ++found;
                }
            }
        }
    }
    if (!pass) counts[k] = found;
}

// ---------------------------------------------------------------- per (block, candidate) waves

// Reduce-scatter of 16 per-lane values over the wave: on return lane l holds
// the wave total of value l >> 2 (17 exchanges instead of 16 x 6).
__device__ __forceinline__ float wave_reduce_scatter16(const float *a, int lane) {
    float b8[8], b4[4], b2[2];
    const bool h5 = lane & 32, h4 = lane & 16, h3 = lane & 8, h2 = lane & 4;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        const float keep = h5 ? a[k + 8] : a[k], send = h5 ? a[k] : a[k + 8];
        b8[k] = keep + __shfl_xor(send, 32, 64);
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const float keep = h4 ? b8[k + 4] : b8[k], send = h4 ? b8[k] : b8[k + 4];
        b4[k] = keep + __shfl_xor(send, 16, 64);
    }
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        const float keep = h3 ? b4[k + 2] : b4[k], send = h3 ? b4[k] : b4[k + 2];
        b2[k] = keep + __shfl_xor(send, 8, 64);
    }
    const float keep = h2 ? b2[1] : b2[0], send = h2 ? b2[0] : b2[1];
    float v = keep + __shfl_xor(send, 4, 64);
    v += __shfl_xor(v, 2, 64);
    v += __shfl_xor(v, 1, 64);
    return v;
}

__device__ __forceinline__ float wave_min_f(float v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fminf(v, __shfl_xor(v, o, 64));
    return v;
}

constexpr int kSup = 16;    // 64-row chunks of detected spots held per lane

// Squared zero radius of a model spot at threshold T (INFINITY where the
// bound does not apply): R_j of the refinement passes' cell marking (see k_single_acc).
__device__ __forceinline__ float zero_radius2(float vv, float vn, float K, float T) {
    const float vn2 = vn * vn;
    const float t2 = 2.0f * (T / K) * vv / vn2;
    if (vn2 >= 1e-4f * vv && t2 < 0.81f) {
        const float t0 = sqrtf(t2);
        const float R = fmaf(t0 * sqrtf(vv) / (1.0f - t0), 1.001f, 1e-3f);
        return R * R;
    }
    return INFINITY;
}

// Whether some lane's detected spot p lies within R (R2 = R^2) of the model
// spot s on the detector (wave-uniform).
__device__ __forceinline__ bool reaches(float p1, float p2, float s1, float s2, float R2) {
    const float dy = p1 - s1, dz = p2 - s2;
    return __any(fmaf(dz, dz, dy * dy) < R2);
}

// Cell index of the detected spots for the refinement passes: each block's
// spots sorted (stably) into a kCellG x kCellG grid over their bounding box,
// so that a pass reads only the cells within reach of a candidate's model
// spots.  Runs of consecutive active cells are contiguous in that order.
constexpr int kCellG = 32;
constexpr int kCells = kCellG * kCellG;
constexpr int kMaxRuns = 256;

// The per-model-spot pass walks a finer grid over the same boxes (cells a
// quarter of the side), so that the cells under a small zero disk hold few
// spots beyond it.
constexpr int kFineG = 128;
constexpr int kFineCells = kFineG * kFineG;

// Cell of a coordinate in cell units (row or column of a G x G grid).
template <int G = kCellG>
__device__ __forceinline__ int cell_coord(float u) {
    return u >= 0.0f ? min(G - 1, static_cast<int>(fminf(u, static_cast<float>(G)))) : 0;
}
// Exponent (log2 units) beyond which an FP32 plan term exp2(-K c') is 0 for
// any rounding of c' (2^-150 already rounds to 0; the margin covers the cost's
// own rounding, a few ulps relative).  The passes skip pairs beyond a
// threshold T <= kZeroExp2 (laue_score_params.drop_log2).
constexpr float kZeroExp2 = 160.0f;

struct SlotArgs {
    int C;                  // candidates in the batch
    int nb;                 // blocks
    const int64_t *offs;    // [nb * C + 1] model-spot offsets per (block, candidate)
    const float *P1, *P2;
    const int64_t *ooff;    // detected-spot block offsets (device)
    const Col8 *colsE, *colsC;
    const GeomF *geom;
    const float *W;
    int n_planes;
    const GrainF *grains;
    const int *mplane, *mgrain, *mblock;
    // cell index (refinement passes): the spots in cell order, per-(block,
    // cell) start positions [nb * kCells + 1], per-block grid (x0, y0, cx, cy)
    const float *P1s, *P2s;
    const float2 *P12s;     // the same, interleaved
    const float2 *P12f;     // the spots in the order of the fine grid (kFineG)
    const int *rowid_f;     // the detected spot's index of each position of that order
    const int *cell_off_f;  // [nb * kFineCells + 1]
    const int *cell_off;
    const float4 *cbox;
    unsigned long long *evaluated;   // pairs the refinement passes evaluate
};

// Column data of model spot j held by lane j, read by the whole wave with
// readlane (j wave-uniform).
struct LaneCol {
    float s1, s2, v1, v2, vv, vv2, vn;
};

__device__ __forceinline__ LaneCol lane_col(const Col8 *cols, int64_t o0, int nc, int lane) {
    LaneCol c{0.0f, 0.0f, 0.0f, 0.0f, 1.0f, 1.0f, 1.0f};
    if (lane < nc) {
        const Col8 v = cols[o0 + lane];
        c = LaneCol{v.s1, v.s2, v.v1, v.v2, v.vv, v.vv2, v.vn};
    }
    return c;
}

__device__ __forceinline__ float bcast(float v, int j) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), j));
}

__device__ __forceinline__ Col8 col_of(const LaneCol &c, int j) {
    return Col8{bcast(c.s1, j), bcast(c.s2, j), bcast(c.v1, j), bcast(c.v2, j),
                bcast(c.vv, j), bcast(c.vv2, j), bcast(c.vn, j), 0.0f};
}

// Plan term and M-step statistics of one pair when the statistics are taken
// at the E-step geometry itself (the first Gauss-Newton step of a refinement
// iteration): the chord cost's intermediates serve both.  With delta = p - s
// (detector-local), b = v.delta, w = 2 b + |delta|^2, the ray d = v + delta
// has |d|^2 = |v|^2 + w and 1/|d| = rsq(|d|^2); the cost
// c' = |v x delta|^2 / (|v|^2 |d|^2 + (v.d) |v| |d|) (chord_cp's expression
// with sqrt(|v|^2 |d|^2) = |v| |d|), the plan entry Q = exp2(-K c') iz, and
// the statistics of accumulate_stats (whose |d| - |v| numerator is the same
// w).  Adds the statistics when Q > 0.
// The pair's intermediates, formed once: its plan term t = exp2(-K c') (the
// row normaliser's own term) and what the statistics need.
struct PairTerm {
    float dy, dz, w, itau, tau, t;
};

__device__ __forceinline__ PairTerm pair_term(float p1, float p2, const Col8 &c, float vlen, float K) {
    PairTerm q;
    q.dy = p1 - c.s1;
    q.dz = p2 - c.s2;
    const float e = fmaf(q.dz, q.dz, q.dy * q.dy);
    const float bb = fmaf(c.v2, q.dz, c.v1 * q.dy);
    q.w = fmaf(2.0f, bb, e);
    const float dd = c.vv + q.w;
    q.itau = __builtin_amdgcn_rsqf(dd);
    q.tau = dd * q.itau;
    const float x2 = fmaf(c.vv, e, -(bb * bb));
    const float den = fmaf((c.vv + bb) * vlen, q.tau, c.vv * dd);
    q.t = fast_exp2(-K * (x2 * __builtin_amdgcn_rcpf(den)));
    return q;
}

// Statistics of a pair with plan entry Q = t / (row normaliser).
__device__ __forceinline__ void spot_entry_stats(float *a, const PairTerm &pt, const Col8 &c, float vlen, float rn,
                                                 float r1, float r2, float Q) {
    if (!(Q > 0.0f)) return;
    const float dy = pt.dy, dz = pt.dz, w = pt.w, itau = pt.itau, tau = pt.tau;
    const float dl = w * __builtin_amdgcn_rcpf(tau + vlen);
    const float e0 = (-rn * dl) * itau;
    const float e1 = fmaf(-r1, dl, dy) * itau;
    const float e2 = fmaf(-r2, dl, dz) * itau;
    const float h0 = c.vn * itau, h1 = (c.v1 + dy) * itau, h2 = (c.v2 + dz) * itau;
    const float wb = Q * itau, wa = wb * itau;
    const float P00 = fmaf(-h0, h0, 1.0f), P01 = -h0 * h1, P02 = -h0 * h2;
    const float P11 = fmaf(-h1, h1, 1.0f), P12 = -h1 * h2, P22 = fmaf(-h2, h2, 1.0f);
    a[0] += Q;
    a[1] = fmaf(Q, e0, a[1]);
    a[2] = fmaf(Q, e1, a[2]);
    a[3] = fmaf(Q, e2, a[3]);
    a[4] = fmaf(wa, P00, a[4]);
    a[5] = fmaf(wa, P01, a[5]);
    a[6] = fmaf(wa, P02, a[6]);
    a[7] = fmaf(wa, P11, a[7]);
    a[8] = fmaf(wa, P12, a[8]);
    a[9] = fmaf(wa, P22, a[9]);
    a[10] = fmaf(wb, P00, a[10]);
    a[11] = fmaf(wb, P01, a[11]);
    a[12] = fmaf(wb, P02, a[12]);
    a[13] = fmaf(wb, P11, a[13]);
    a[14] = fmaf(wb, P12, a[14]);
    a[15] = fmaf(wb, P22, a[15]);
}

// Single-grain E-step (row softmax with the outlier column, App. D) fused
// with the M-step statistics: Q from the columns colsE (held fixed over the
// Gauss-Newton steps of one refinement iteration), statistics at the current
// columns colsC.  Writes per (candidate, block) the summed 27-value
// normal-equation contribution.  One wave per (block b, candidate c), item =
// b * C + c so that neighbouring waves stream the same detected spots.  The
// Gauss-Newton steps after the first of an iteration (colsC not colsE; the
// first step runs per model spot, k_spot_acc).  The loops over a lane's kSup
// rows are unrolled with wave-uniform guards, so the rows stay in named
// registers.
__global__ __launch_bounds__(64) void k_single_acc(SlotArgs A, float K, float bin_e, float T_skip,
                                                   double *__restrict__ st_out) {
    const int item = blockIdx.x;
    const int b = item / A.C, c = item - b * A.C;
    const int lane = threadIdx.x;
    const int64_t o0 = A.offs[static_cast<int64_t>(b) * A.C + c];
    const int nc = static_cast<int>(A.offs[static_cast<int64_t>(b) * A.C + c + 1] - o0);
    const int64_t r0 = A.ooff[b], rend = A.ooff[b + 1];
    if (nc == 0) return;
    const LaneCol lE = lane_col(A.colsE, o0, nc, lane);
    const LaneCol lC = lane_col(A.colsC, o0, nc, lane);
    // per-column constants at the current geometry: |v|, v / |v|
    const float ivl_l = __builtin_amdgcn_rsqf(lC.vv), vlen_l = lC.vv * ivl_l;
    const float rn_l = lC.vn * ivl_l, r1_l = lC.v1 * ivl_l, r2_l = lC.v2 * ivl_l;
    // FP64 running statistics of model spot j at acc[16 j + q] (this wave only)
    __shared__ double acc[64 * kStat];
    for (int k = lane; k < nc * kStat; k += 64) acc[k] = 0.0;
    // the columns' constants in LDS, read back by every lane with one
    // broadcast load per value: the pair arithmetic then takes vector-register
    // operands only (a scalar-register operand halves the VALU issue rate)
    __shared__ float4 cst[64 * 5];
    if (lane < nc) {
        cst[lane] = make_float4(lE.s1, lE.s2, lE.v1, lE.v2);
        cst[64 + lane] = make_float4(lE.vv, lE.vv2, lE.vn, vlen_l);
        cst[128 + lane] = make_float4(rn_l, r1_l, r2_l, 0.0f);
        cst[192 + lane] = make_float4(lC.s1, lC.s2, lC.v1, lC.v2);
        cst[256 + lane] = make_float4(lC.vv, lC.vv2, lC.vn, 0.0f);
    }
    // Rows that can carry weight.  Every plan term of model spot j has
    // exponent K c' >= T_skip (so is 0 in FP32 for T_skip = kZeroExp2, or
    // below 2^-drop_log2 of the outlier bin's term) for detected spots
    // farther than R_j from s_j on the detector: with delta = p - s in the
    // detector plane and v_n the normal part of v, |v x delta| >= |delta| v_n
    // and |v|^2 |d|^2 + (v.d)|v||d| <= 2 |v|^2 (|v| + |delta|)^2, so
    // c' >= t^2 v_n^2 / (2 |v|^2) with t = |delta| / (|v| + |delta|), and
    // K c' >= T_skip once t >= t0 = sqrt(2 T_skip |v|^2 / (K v_n^2)),
    // i.e. |delta| >= R_j = t0 |v| / (1 - t0).  The cells of the block's grid
    // within R_j of some s_j are marked; their spots, in cell order, are the
    // rows of the passes below (all of the block's when the marked cells
    // hold most of them or form too many runs).
    __shared__ float rad2[64];
    __shared__ unsigned cmask[kCells / 32];
    __shared__ int run_at[kMaxRuns], run_pre[kMaxRuns + 1];
    rad2[lane] = lane < nc ? zero_radius2(lE.vv, lE.vn, K, T_skip) : INFINITY;
    if (lane < kCells / 32) cmask[lane] = 0u;
    __syncthreads();
    const float4 bx = A.cbox[b];   // x0, y0, cx, cy
    const float pad_x = 1e-3f * bx.z + 1e-4f, pad_y = 1e-3f * bx.w + 1e-4f;
    for (int j = 0; j < nc; ++j) {
        const float R2 = rad2[j], s1 = cst[j].x, s2 = cst[j].y;
        int ix0 = 0, ix1 = kCellG - 1, iy0 = 0, iy1 = kCellG - 1;
        if (R2 < INFINITY) {
            const float R = sqrtf(R2);
            // cell coordinates clamped to [-2, 2 G] before the conversion
            const float lo = -2.0f, hi = 2.0f * kCellG;
            ix0 = max(0, static_cast<int>(floorf(fminf(fmaxf((s1 - R - bx.x) / bx.z, lo), hi))) - 1);
            ix1 = min(kCellG - 1, static_cast<int>(floorf(fminf(fmaxf((s1 + R - bx.x) / bx.z, lo), hi))) + 1);
            iy0 = max(0, static_cast<int>(floorf(fminf(fmaxf((s2 - R - bx.y) / bx.w, lo), hi))) - 1);
            iy1 = min(kCellG - 1, static_cast<int>(floorf(fminf(fmaxf((s2 + R - bx.y) / bx.w, lo), hi))) + 1);
        }
        const int wdt = ix1 - ix0 + 1, hgt = iy1 - iy0 + 1;
        if (wdt <= 0 || hgt <= 0) continue;
        for (int k = lane; k < wdt * hgt; k += 64) {
            const int ix = ix0 + k % wdt, iy = iy0 + k / wdt;
            const float xa = fmaf(static_cast<float>(ix), bx.z, bx.x) - pad_x, xb = xa + bx.z + 2.0f * pad_x;
            const float ya = fmaf(static_cast<float>(iy), bx.w, bx.y) - pad_y, yb = ya + bx.w + 2.0f * pad_y;
            const float dx = fmaxf(0.0f, fmaxf(xa - s1, s1 - xb)), dy = fmaxf(0.0f, fmaxf(ya - s2, s2 - yb));
            if (fmaf(dx, dx, dy * dy) < R2) {
                const int cell = iy * kCellG + ix;
                atomicOr(&cmask[cell >> 5], 1u << (cell & 31));
            }
        }
    }
    __syncthreads();
    // runs of marked cells: lane l takes cells 16 l .. 16 l + 15
    const int *co = A.cell_off + static_cast<int64_t>(b) * kCells;
    int n_runs, n_act;
    {
        const unsigned bits = (cmask[lane >> 1] >> ((lane & 1) * 16)) & 0xFFFFu;
        const unsigned starts = bits & ~(bits << 1);
        const int my_runs = __popc(starts);
        int my_rows = 0;
        for (unsigned st = starts; st; st &= st - 1) {
            const int c0 = __ffs(st) - 1;
            int c1 = c0;
            while (c1 + 1 < 16 && ((bits >> (c1 + 1)) & 1u)) ++c1;
            my_rows += co[16 * lane + c1 + 1] - co[16 * lane + c0];
        }
        int run_base = my_runs, row_base = my_rows;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const int a1 = __shfl_up(run_base, o, 64), a2 = __shfl_up(row_base, o, 64);
            if (lane >= o) {
                run_base += a1;
                row_base += a2;
            }
        }
        n_runs = __shfl(run_base, 63, 64);
        n_act = __shfl(row_base, 63, 64);
        run_base -= my_runs;
        row_base -= my_rows;
        const int n_block = static_cast<int>(rend - r0);
        if (n_runs > kMaxRuns || 4 * n_act > 3 * n_block) {
            n_runs = 1;
            n_act = n_block;
            if (lane == 0) {
                run_at[0] = static_cast<int>(r0);
                run_pre[0] = 0;
            }
        } else {
            int k = run_base, pre = row_base;
            for (unsigned st = starts; st; st &= st - 1) {
                const int c0 = __ffs(st) - 1;
                int c1 = c0;
                while (c1 + 1 < 16 && ((bits >> (c1 + 1)) & 1u)) ++c1;
                run_at[k] = co[16 * lane + c0];
                run_pre[k] = pre;
                pre += co[16 * lane + c1 + 1] - co[16 * lane + c0];
                ++k;
            }
        }
        if (lane == 0) run_pre[n_runs] = n_act;
    }
    if (lane == 0 && n_act > 0 && A.evaluated)
        atomicAdd(A.evaluated, static_cast<unsigned long long>(n_act) * static_cast<unsigned long long>(nc));
    __syncthreads();
    // Those rows in super-chunks of kSup x 64: each lane keeps its kSup rows
    // (coordinates and softmax normalisers) in registers, so the statistics
    // of a model spot accumulate per lane over the whole super-chunk and are
    // wave-reduced once per super-chunk.
    int kr = 0;   // this lane's current run
    for (int s0 = 0; s0 < n_act; s0 += 64 * kSup) {
        const int nrow = min(64 * kSup, n_act - s0);
        float p1[kSup], p2[kSup], iz[kSup];
#pragma unroll
        for (int u = 0; u < kSup; ++u) {
            const int pos = s0 + 64 * u + lane;
            const bool rv = pos < n_act;
            while (rv && kr + 1 < n_runs && run_pre[kr + 1] <= pos) ++kr;
            const int row = rv ? run_at[kr] + (pos - run_pre[kr]) : static_cast<int>(r0);
            p1[u] = rv ? A.P1s[row] : 0.0f;
            p2[u] = rv ? A.P2s[row] : 0.0f;
            iz[u] = bin_e;
        }
        // a 64-row chunk none of whose rows lies within R_j of s_j adds
        // terms below the threshold only: it skips model spot j
        for (int j = 0; j < nc; ++j) {
            const float4 x0 = cst[j], x1 = cst[64 + j];
            const float R2 = rad2[j];
#pragma unroll
            for (int u = 0; u < kSup; ++u)
                if (64 * u < nrow && reaches(p1[u], p2[u], x0.x, x0.y, R2))
                    iz[u] += fast_exp2(entry_exponent(p1[u], p2[u], x0.x, x0.y, x0.z, x0.w, x1.x, x1.y, K, 0.0f));
        }
#pragma unroll
        for (int u = 0; u < kSup; ++u) iz[u] = 64 * u + lane < nrow ? __builtin_amdgcn_rcpf(iz[u]) : 0.0f;
        for (int j = 0; j < nc; ++j) {
            const float4 x0 = cst[j], x1 = cst[64 + j], x2 = cst[128 + j];
            const Col8 cE{x0.x, x0.y, x0.z, x0.w, x1.x, x1.y, x1.z, 0.0f};
            const float vl = x1.w, rn = x2.x, r1 = x2.y, r2 = x2.z;
            const float R2 = rad2[j];
            float a[kStat];
#pragma unroll
            for (int q = 0; q < kStat; ++q) a[q] = 0.0f;
            bool any = false;
            const float4 y0 = cst[192 + j], y1 = cst[256 + j];
            const Col8 cC{y0.x, y0.y, y0.z, y0.w, y1.x, y1.y, y1.z, 0.0f};
#pragma unroll
            for (int u = 0; u < kSup; ++u) {
                if (64 * u < nrow && reaches(p1[u], p2[u], cE.s1, cE.s2, R2)) {
                    const float Q = fast_exp2(entry_exponent(p1[u], p2[u], cE.s1, cE.s2, cE.v1, cE.v2, cE.vv,
                                                             cE.vv2, K, 0.0f)) *
                                    iz[u];
                    if (__any(Q > 0.0f)) {                      // weight in this chunk
                        any = true;
                        accumulate_stats(a, Q, p1[u], p2[u], cC, vl, rn, r1, r2);   // Q = 0 adds zeros
                    }
                }
            }
            if (!any) continue;
            const float t = wave_reduce_scatter16(a, lane);
            if ((lane & 3) == 0) acc[kStat * j + (lane >> 2)] += static_cast<double>(t);
        }
    }
    __syncthreads();
    // the model spots' statistics; k_single_normal forms their normal equations
    if (lane < nc) {
        double *dst = st_out + (o0 + lane) * kStat;
#pragma unroll
        for (int q = 0; q < kStat; ++q) dst[q] = acc[kStat * lane + q];
    }
}

// One wave per candidate: the FP64 normal equations of each of its model
// spots from the statistics of k_single_acc (lane l takes the spots of blocks
// l, l + 64, ...; the current columns colsC give the spot's unit ray), summed
// over the wave in a fixed order into hg[c] (kHg values).
__global__ __launch_bounds__(64) void k_single_normal(SlotArgs A, const double *__restrict__ st, double D2,
                                                      double *__restrict__ hg_out) {
    const int c = blockIdx.x;
    if (c >= A.C) return;
    double acc[kHg];
    for (int k = 0; k < kHg; ++k) acc[k] = 0.0;
    for (int b = threadIdx.x; b < A.nb; b += 64) {
        const int64_t o1 = A.offs[static_cast<int64_t>(b) * A.C + c + 1];
        for (int64_t o = A.offs[static_cast<int64_t>(b) * A.C + c]; o < o1; ++o) {
            const Col8 cc = A.colsC[o];
            const float ivl = __builtin_amdgcn_rsqf(cc.vv);
            double s64[kStat], hg[kHg];
            for (int k = 0; k < kStat; ++k) s64[k] = st[o * kStat + k];
            column_normal_equations(*A.geom, A.W, A.n_planes, A.grains, A.C, A.mplane[o], A.mgrain[o],
                                    A.mblock[o], s64, cc.vn * ivl, cc.v1 * ivl, cc.v2 * ivl, D2, hg);
            for (int k = 0; k < kHg; ++k) acc[k] += hg[k];
        }
    }
    for (int k = 0; k < kHg; ++k) acc[k] = wave_sum(acc[k]);
    if (threadIdx.x != 0) return;
    double *dst = hg_out + static_cast<int64_t>(c) * kHg;
    for (int k = 0; k < kHg; ++k) dst[k] = acc[k];
}

// One thread per candidate: the Gauss-Newton step from its summed normal
// equations (64 candidates' factorisations side by side in a wave).
__global__ __launch_bounds__(64) void k_single_step(int C, const double *__restrict__ hg, double mu_rel, double *q,
                                                    double *x, GrainF *__restrict__ gf) {
    const int c = blockIdx.x * 64 + threadIdx.x;
    if (c >= C) return;
    gn_solve_apply(hg + static_cast<int64_t>(c) * kHg, mu_rel, q + 4 * c, x + 3 * c, gf + c, nullptr);
}

// ---------------------------------------------------------------- per model spot refinement pass

// The (block, candidate) slot of model spot o: [*o0, *o1) and its block
// (and, if item is given, block * C + candidate).
__device__ __forceinline__ int spot_slot(const SlotArgs &A, int64_t o, int64_t *o0, int64_t *o1,
                                         int64_t *item_out = nullptr) {
    int b = A.mblock[o];
    const int g = A.mgrain[o];
    int64_t item = static_cast<int64_t>(b) * A.C + g;
    if (b < 0 || b >= A.nb || g < 0 || g >= A.C || !(A.offs[item] <= o && o < A.offs[item + 1])) {
        // by the offsets themselves
        int64_t lo = 0, hi = static_cast<int64_t>(A.nb) * A.C - 1;
        while (lo < hi) {
            const int64_t mid = (lo + hi + 1) >> 1;
            if (A.offs[mid] <= o) lo = mid;
            else hi = mid - 1;
        }
        item = lo;
        b = static_cast<int>(item / A.C);
    }
    *o0 = A.offs[item];
    *o1 = A.offs[item + 1];
    if (item_out) *item_out = item;
    return b;
}

__global__ void k_spot_rad(const Col8 *__restrict__ cols, int64_t M, float K, float T, float *__restrict__ rad2) {
    for (int64_t o = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; o < M;
         o += static_cast<int64_t>(gridDim.x) * blockDim.x)
        rad2[o] = zero_radius2(cols[o].vv, cols[o].vn, K, T);
}

// Bit k of nbr[o]: model spot o0 + k of o's slot has a zero disk that meets
// o's (its own bit included): only those can weigh on a row within reach of o.
__global__ void k_spot_nbr(SlotArgs A, const float *__restrict__ rad2, int64_t M,
                           unsigned long long *__restrict__ nbr) {
    for (int64_t o = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; o < M;
         o += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        int64_t o0, o1;
        spot_slot(A, o, &o0, &o1);
        const float Ro = sqrtf(rad2[o]);
        const float s1 = A.colsE[o].s1, s2 = A.colsE[o].s2;
        unsigned long long m = 0ull;
        for (int64_t j = o0; j < o1; ++j) {
            const float R = Ro + sqrtf(rad2[j]);
            const float dy = A.colsE[j].s1 - s1, dz = A.colsE[j].s2 - s2;
            if (j == o || !(fmaf(dz, dz, dy * dy) >= R * R)) m |= 1ull << (j - o0);
        }
        nbr[o] = m;
    }
}

// The statistics pass of the first Gauss-Newton step of a refinement
// iteration (statistics at the E-step geometry colsE), one thread per model
// spot o: the detected spots of the cell rows of o's cell
// box, those within R_o of s_o, each with its row normaliser (the bin term,
// then the terms of the slot's spots that reach the row, in index order: a
// spot out of reach adds less than a quarter ulp, so the normaliser is the
// one over every spot of the slot; o's own term is the one its statistics
// use), accumulated in FP32 over 16 rows at a time and in FP64 across.
// Writes o's kStat statistics.
__global__ __launch_bounds__(256) void k_spot_acc(SlotArgs A, float K, float bin_e, const float *__restrict__ rad2,
                                                  const unsigned long long *__restrict__ nbr, int64_t M,
                                                  double *__restrict__ st_out) {
    const int64_t o = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    unsigned long long evaluated = 0;
    if (o < M) {
        int64_t o0, o1;
        const int b = spot_slot(A, o, &o0, &o1);
        const Col8 me = A.colsE[o];
        const float R2 = rad2[o];
        const unsigned long long mask = nbr[o];
        const float ivl = __builtin_amdgcn_rsqf(me.vv), vl = me.vv * ivl;
        const float rn = me.vn * ivl, r1 = me.v1 * ivl, r2 = me.v2 * ivl;
        double acc[kStat];
        float a[kStat];
#pragma unroll
        for (int q = 0; q < kStat; ++q) {
            acc[q] = 0.0;
            a[q] = 0.0f;
        }
        // the cells a spot within R_o can fall in (cell_coord of the
        // coordinate range, widened by a thousandth of a cell against the
        // rounding of the cell assignment), per cell row the chord of the
        // disk over that row's band
        const float4 bc = A.cbox[b];
        const float4 bx = make_float4(bc.x, bc.y, bc.z * (static_cast<float>(kCellG) / kFineG),
                                      bc.w * (static_cast<float>(kCellG) / kFineG));
        // hardware sqrt and reciprocal (an ulp or two): the ranges are
        // widened by eps_c cells, far beyond that; the reach test below is
        // exact
        const float R = __builtin_amdgcn_sqrtf(R2);
        const float eps_c = 1e-3f;
        const float icx = __builtin_amdgcn_rcpf(bx.z), icy = __builtin_amdgcn_rcpf(bx.w);
        const int iy0 = cell_coord<kFineG>((me.s2 - R - bx.y) * icy - eps_c);
        const int iy1 = cell_coord<kFineG>((me.s2 + R - bx.y) * icy + eps_c);
        const int *co = A.cell_off_f + static_cast<int64_t>(b) * kFineCells;
        int n16 = 0;
        for (int iy = iy0; iy <= iy1; ++iy) {
            const float ya = bx.y + (static_cast<float>(iy) - eps_c) * bx.w;
            const float yb = bx.y + (static_cast<float>(iy + 1) + eps_c) * bx.w;
            const float dyb = fmaxf(0.0f, fmaxf(ya - me.s2, me.s2 - yb));
            if (!(dyb * dyb < R2)) continue;
            const float hw = __builtin_amdgcn_sqrtf(R2 - dyb * dyb);
            const int ix0 = cell_coord<kFineG>((me.s1 - hw - bx.x) * icx - eps_c);
            const int ix1 = cell_coord<kFineG>((me.s1 + hw - bx.x) * icx + eps_c);
            const int re = co[iy * kFineG + ix1 + 1];
            // four rows' loads in flight before the first is used
            for (int r0 = co[iy * kFineG + ix0]; r0 < re; r0 += 4) {
                float2 pq[4];
#pragma unroll
                for (int u = 0; u < 4; ++u)
                    pq[u] = r0 + u < re ? A.P12f[r0 + u] : make_float2(INFINITY, INFINITY);
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                const float p1 = pq[u].x, p2 = pq[u].y;
                const float dy = p1 - me.s1, dz = p2 - me.s2;
                if (!(fmaf(dz, dz, dy * dy) < R2)) continue;
                ++evaluated;
                const PairTerm pt = pair_term(p1, p2, me, vl, K);
                float z = bin_e;
                for (unsigned long long m = mask; m; m &= m - 1) {
                    const int64_t j = o0 + __builtin_ctzll(m);
                    if (j == o) {
                        z += pt.t;
                    } else {
                        const Col8 cj = A.colsE[j];
                        const float ey = p1 - cj.s1, ez = p2 - cj.s2;
                        if (fmaf(ez, ez, ey * ey) < rad2[j])
                            z += fast_exp2(entry_exponent(p1, p2, cj.s1, cj.s2, cj.v1, cj.v2, cj.vv, cj.vv2, K,
                                                          0.0f));
                    }
                }
                spot_entry_stats(a, pt, me, vl, rn, r1, r2, pt.t * __builtin_amdgcn_rcpf(z));
                if (++n16 == 16) {
#pragma unroll
                    for (int q = 0; q < kStat; ++q) {
                        acc[q] += static_cast<double>(a[q]);
                        a[q] = 0.0f;
                    }
                    n16 = 0;
                }
                }
            }
        }
        double *dst = st_out + o * kStat;
#pragma unroll
        for (int q = 0; q < kStat; ++q) dst[q] = acc[q] + static_cast<double>(a[q]);
    }
    if (A.evaluated) {
        for (int off = 32; off > 0; off >>= 1)
            evaluated += __shfl_xor(evaluated, off, 64);
        if ((threadIdx.x & 63) == 0 && evaluated) atomicAdd(A.evaluated, evaluated);
    }
}

// Scoring radius of each model spot o (at the scoring geometry colsC, nc
// spots in its slot): beyond it every row's cost to o exceeds c_out (the
// unmatched test), and o's term of a row's sum is below floor_e / (2 nc), so
// a row beyond the radius of every spot of the slot sums to less than half the
// floor (no SPOT entry).  Lhit = -log2(floor_e).
__global__ void k_score_rad(SlotArgs A, int64_t M, float twoD2, float K2, float c_out, float Lhit,
                            float *__restrict__ rad2) {
    for (int64_t o = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; o < M;
         o += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        int64_t o0, o1;
        spot_slot(A, o, &o0, &o1);
        const Col8 c = A.colsC[o];
        const float Thit = Lhit + 1.0f + log2f(static_cast<float>(o1 - o0));
        rad2[o] = fmaxf(zero_radius2(c.vv, c.vn, twoD2, c_out * 1.001f), zero_radius2(c.vv, c.vn, K2, Thit));
    }
}

// The scoring passes at the final grains (colsC), one thread per model spot
// o over the detected spots within its scoring radius (the fine cell grid, as
// in k_spot_acc).  Unmatched: no detected spot with 2 D^2 c' <= c_out (the
// spots beyond the radius are all farther).  SPOT entry of a detected spot
// and candidate: Lbar = ln sum_j exp2(-K2 c'_j) over the candidate's model
// spots j of the block, in index order, when the sum exceeds floor_e; a row
// is taken by the lowest-index spot of the slot whose radius holds it (rows
// beyond every radius have no entry).  pass 0 counts o's entries (hcnt) and
// adds them and o's unmatched flag to its (candidate, block) slot (unm and
// lcnt start at zero); pass 1 writes the kept candidates' entries at loff of
// the slot plus the counts of the slot's earlier spots, in o's walk order
// (CSR by candidate, then block).  Lrow is the detected spot's index.
template <int PASS>
__global__ __launch_bounds__(256) void k_spot_score(SlotArgs A, int64_t M, float twoD2, float K2, float floor_e,
                                                    float c_out, const float *__restrict__ rad2,
                                                    const unsigned long long *__restrict__ nbr, int *__restrict__ hcnt,
                                                    int *__restrict__ unm, int *__restrict__ lcnt,
                                                    const int64_t *__restrict__ loff,
                                                    const uint8_t *__restrict__ keep, int *__restrict__ lrow,
                                                    float *__restrict__ lval, unsigned long long *ev) {
    const int64_t o = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    unsigned long long evaluated = 0;
    int64_t o0 = 0, o1 = 0, item = 0;
    if (o < M) spot_slot(A, o, &o0, &o1, &item);
    const int b = static_cast<int>(item / A.C), c = static_cast<int>(item - static_cast<int64_t>(b) * A.C);
    const int64_t slot = static_cast<int64_t>(c) * A.nb + b;
    if (o < M && (PASS == 0 || keep[c])) {
        const Col8 me = A.colsC[o];
        const float R2 = rad2[o];
        // the slot's spots before o whose radius may hold a row within o's
        const unsigned long long before = nbr[o] & ((1ull << (o - o0)) - 1ull);
        int64_t pos = 0;
        if (PASS == 1) {
            pos = loff[slot];
            for (int64_t j = o0; j < o; ++j) pos += hcnt[j];
        }
        bool matched = false;
        int h = 0;
        const float4 bc = A.cbox[b];
        const float4 bx = make_float4(bc.x, bc.y, bc.z * (static_cast<float>(kCellG) / kFineG),
                                      bc.w * (static_cast<float>(kCellG) / kFineG));
        const float R = __builtin_amdgcn_sqrtf(R2);
        const float eps_c = 1e-3f;
        const float icx = __builtin_amdgcn_rcpf(bx.z), icy = __builtin_amdgcn_rcpf(bx.w);
        const int iy0 = cell_coord<kFineG>((me.s2 - R - bx.y) * icy - eps_c);
        const int iy1 = cell_coord<kFineG>((me.s2 + R - bx.y) * icy + eps_c);
        const int *co = A.cell_off_f + static_cast<int64_t>(b) * kFineCells;
        for (int iy = iy0; iy <= iy1; ++iy) {
            const float ya = bx.y + (static_cast<float>(iy) - eps_c) * bx.w;
            const float yb = bx.y + (static_cast<float>(iy + 1) + eps_c) * bx.w;
            const float dyb = fmaxf(0.0f, fmaxf(ya - me.s2, me.s2 - yb));
            if (!(dyb * dyb < R2)) continue;
            const float hw = __builtin_amdgcn_sqrtf(R2 - dyb * dyb);
            const int ix0 = cell_coord<kFineG>((me.s1 - hw - bx.x) * icx - eps_c);
            const int ix1 = cell_coord<kFineG>((me.s1 + hw - bx.x) * icx + eps_c);
            const int re = co[iy * kFineG + ix1 + 1];
            for (int r = co[iy * kFineG + ix0]; r < re; ++r) {
                const float2 pq = A.P12f[r];
                const float p1 = pq.x, p2 = pq.y;
                const float dy = p1 - me.s1, dz = p2 - me.s2;
                if (!(fmaf(dz, dz, dy * dy) < R2)) continue;
                if (PASS == 0 && !matched) {
                    const float cp = entry_exponent(p1, p2, me.s1, me.s2, me.v1, me.v2, me.vv, me.vv2, -1.0f, 0.0f);
                    matched = twoD2 * cp <= c_out;
                }
                bool own = true;
                for (unsigned long long m = before; m; m &= m - 1) {
                    const int64_t j = o0 + __builtin_ctzll(m);
                    const Col8 cj = A.colsC[j];
                    const float ey = p1 - cj.s1, ez = p2 - cj.s2;
                    if (fmaf(ez, ez, ey * ey) < rad2[j]) {
                        own = false;
                        break;
                    }
                }
                if (!own) continue;
                float zz = 0.0f;
                for (int64_t j = o0; j < o1; ++j) {
                    const Col8 cj = A.colsC[j];
                    const float cp = entry_exponent(p1, p2, cj.s1, cj.s2, cj.v1, cj.v2, cj.vv, cj.vv2, -1.0f, 0.0f);
                    zz += fast_exp2(-K2 * cp);
                }
                evaluated += static_cast<unsigned long long>(o1 - o0);
                if (zz > floor_e) {
                    if (PASS == 0) {
                        ++h;
                    } else {
                        lrow[pos] = A.rowid_f[r];
                        lval[pos] = __logf(zz);
                        ++pos;
                    }
                }
            }
        }
        if (PASS == 0) {
            hcnt[o] = h;
            if (h) atomicAdd(&lcnt[slot], h);
            if (!matched) atomicAdd(&unm[slot], 1);
        }
    }
    if (ev) {
        for (int off = 32; off > 0; off >>= 1)
            evaluated += __shfl_xor(evaluated, off, 64);
        if ((threadIdx.x & 63) == 0 && evaluated) atomicAdd(ev, evaluated);
    }
}

__global__ void k_fill_int2(int *__restrict__ a, int *__restrict__ b, int64_t n) {
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
         i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        a[i] = 0;
        b[i] = 0;
    }
}

// Keep decision per candidate: unmatched fraction < f_out (Sec. 6.2, Sec. 7).
// Dropped candidates get no SPOT entries.
__global__ void k_single_keep(int C, int nb, const int64_t *__restrict__ offs,
                              const int *__restrict__ unm, int *__restrict__ lcnt, double f_out,
                              uint8_t *__restrict__ keep_ws, int *__restrict__ o_nmodel,
                              int *__restrict__ o_unm, uint8_t *__restrict__ o_keep) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= C) return;
    int64_t nm = 0, nu = 0;
    for (int b = 0; b < nb; ++b) {
        nm += offs[static_cast<int64_t>(b) * C + c + 1] - offs[static_cast<int64_t>(b) * C + c];
        nu += unm[static_cast<int64_t>(c) * nb + b];
    }
    const bool keep = nm > 0 && static_cast<double>(nu) < f_out * static_cast<double>(nm);
    if (!keep)
        for (int b = 0; b < nb; ++b) lcnt[static_cast<int64_t>(c) * nb + b] = 0;
    keep_ws[c] = keep ? 1 : 0;
    if (o_nmodel) o_nmodel[c] = static_cast<int>(nm);
    if (o_unm) o_unm[c] = static_cast<int>(nu);
    if (o_keep) o_keep[c] = keep ? 1 : 0;
}

__global__ void k_max_int(const int *__restrict__ v, int64_t n, int *__restrict__ out) {
    __shared__ int part[256];
    int m = 0;
    for (int64_t i = threadIdx.x; i < n; i += 256) m = max(m, v[i]);
    part[threadIdx.x] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        int r = 0;
        for (int k = 0; k < 256; ++k) r = max(r, part[k]);
        *out = r;
    }
}

// cand_off[c0 + c] = base + loff[c * nb] for the batch's candidates.
__global__ void k_cand_off(const int64_t *__restrict__ loff, int C, int nb, int64_t base,
                           int64_t *__restrict__ cand_off, int c0, int last) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c < C) cand_off[c0 + c] = base + loff[static_cast<int64_t>(c) * nb];
    if (last && c == C) cand_off[c0 + C] = base + loff[static_cast<int64_t>(C) * nb];
}

// ---------------------------------------------------------------- SPOT greedy

// One lane's part of a candidate's increment: entries lane, lane + 64, ...
// of its CSR range [e0, e1), added in that order (four loads in flight per
// step, the order unchanged), so every caller gets the same value bit for bit.
__device__ __forceinline__ double lane_gain(int64_t e0, int64_t e1, int lane, const int *__restrict__ row,
                                            const float *__restrict__ val, const float *__restrict__ cur) {
    double s = 0.0;
    int64_t e = e0 + lane;
    for (; e + 192 < e1; e += 256) {
        const int r0 = row[e], r1 = row[e + 64], r2 = row[e + 128], r3 = row[e + 192];
        const float v0 = val[e], v1 = val[e + 64], v2 = val[e + 128], v3 = val[e + 192];
        const float c0 = cur[r0], c1 = cur[r1], c2 = cur[r2], c3 = cur[r3];
        s += fmax(0.0, static_cast<double>(v0) - static_cast<double>(c0));
        s += fmax(0.0, static_cast<double>(v1) - static_cast<double>(c1));
        s += fmax(0.0, static_cast<double>(v2) - static_cast<double>(c2));
        s += fmax(0.0, static_cast<double>(v3) - static_cast<double>(c3));
    }
    for (; e < e1; e += 64) s += fmax(0.0, static_cast<double>(val[e]) - static_cast<double>(cur[row[e]]));
    return s;
}

// lane_gain over the lane's positions of [e0, e0 + L) that also moves the
// lane's live entries (Lbar above the row's cover) down to its first
// positions e0 + lane + 64 k, in order: the entries it drops add exactly 0
// to this and every later increment (covers only rise), so a lane's FP64 sum
// over the kept entries is the sum over all of them bit for bit.  n_live
// returns the lane's kept entries.
__device__ __forceinline__ double lane_gain_compact(int64_t e0, int64_t L, int lane, int *row, float *val,
                                                    const float *__restrict__ cur, int &n_live) {
    double s = 0.0;
    int n = 0;
    int64_t e = e0 + lane;
    const int64_t e1 = e0 + L;
    auto keep = [&](int64_t at, int r, float v, float c) {
        if (v > c) {
            const int64_t d = e0 + lane + 64 * static_cast<int64_t>(n);
            if (d != at) {
                row[d] = r;
                val[d] = v;
            }
            ++n;
        }
    };
    for (; e + 192 < e1; e += 256) {
        const int r0 = row[e], r1 = row[e + 64], r2 = row[e + 128], r3 = row[e + 192];
        const float v0 = val[e], v1 = val[e + 64], v2 = val[e + 128], v3 = val[e + 192];
        const float c0 = cur[r0], c1 = cur[r1], c2 = cur[r2], c3 = cur[r3];
        s += fmax(0.0, static_cast<double>(v0) - static_cast<double>(c0));
        s += fmax(0.0, static_cast<double>(v1) - static_cast<double>(c1));
        s += fmax(0.0, static_cast<double>(v2) - static_cast<double>(c2));
        s += fmax(0.0, static_cast<double>(v3) - static_cast<double>(c3));
        keep(e, r0, v0, c0);
        keep(e + 64, r1, v1, c1);
        keep(e + 128, r2, v2, c2);
        keep(e + 192, r3, v3, c3);
    }
    for (; e < e1; e += 64) {
        const int r = row[e];
        const float v = val[e], c = cur[r];
        s += fmax(0.0, static_cast<double>(v) - static_cast<double>(c));
        keep(e, r, v, c);
    }
    n_live = n;
    return s;
}

__global__ __launch_bounds__(64) void k_gain(const int64_t *__restrict__ off,
                                             const int *__restrict__ row,
                                             const float *__restrict__ val,
                                             const float *__restrict__ cur,
                                             const uint8_t *__restrict__ picked,
                                             double *__restrict__ gain, const int *__restrict__ done,
                                             int n) {
    const int c = blockIdx.x;
    if (c >= n || *done) return;
    if (picked[c]) {
        if (threadIdx.x == 0) gain[c] = -1.0;
        return;
    }
    const double s = wave_sum(lane_gain(off[c], off[c + 1], static_cast<int>(threadIdx.x), row, val, cur));
    if (threadIdx.x == 0) gain[c] = s;
}

// Band steps of the greedy: the same picks and increments as recomputing every
// increment at every step.  An increment can only fall as rows are covered
// (cur only rises), so an increment computed at an earlier step bounds the
// current one from above: ub[c] is such a bound, exact when stamp[c] is the
// current step.  A step scans every unpicked candidate for the best exact
// increment (lowest index on ties) and the largest stale bound S; when the
// best exact increment is positive and above S it is the exact argmax and is
// picked.  Otherwise the stale bounds at or above a threshold are recomputed
// grid-wide and the scan repeats: first the threshold S (the candidates of the
// largest bound), then the best exact increment so found, after which no stale
// bound reaches the best exact increment and the third scan decides the step
// (no positive exact increment: the selection ends).
constexpr int kBandScanBlocks = 1024;
constexpr int kBandRefreshWaves = 4096;

struct BandState {
    double thr;    // recompute stale bounds >= thr (and > 0)
    int decided;   // last step whose pick is made
};

__global__ void k_band_init(BandState *st) {
    st->thr = 0.0;
    st->decided = -1;
}

// (value, index) maximum, the lower index on equal values; index -1 is empty.
__device__ __forceinline__ void band_best(double &b, int &bi, double ob, int oi) {
    if (oi >= 0 && (bi < 0 || ob > b || (ob == b && oi < bi))) {
        b = ob;
        bi = oi;
    }
}

// Per block: best exact (ub, index) at this step and the largest stale bound.
__global__ __launch_bounds__(256) void k_band_scan(const uint8_t *__restrict__ picked, const double *__restrict__ ub,
                                                   const int *__restrict__ stamp, int n, int step,
                                                   const BandState *__restrict__ st, const int *__restrict__ done,
                                                   double *__restrict__ pb, int *__restrict__ pi,
                                                   double *__restrict__ ps) {
    __shared__ double lb[4], ls[4];
    __shared__ int li[4];
    if (*done || st->decided == step) return;
    double b = -1.0, sm = -1.0;
    int bi = -1;
    for (int c = blockIdx.x * 256 + threadIdx.x; c < n; c += gridDim.x * 256) {
        if (picked[c]) continue;
        const double g = ub[c];
        if (stamp[c] == step) {
            if (bi < 0 || g > b) {   // c ascends: the first of equal values stays
                b = g;
                bi = c;
            }
        } else {
            sm = fmax(sm, g);
        }
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const double ob = __shfl_xor(b, o, 64);
        const int oi = __shfl_xor(bi, o, 64);
        band_best(b, bi, ob, oi);
        sm = fmax(sm, __shfl_xor(sm, o, 64));
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) {
        lb[wave] = b;
        li[wave] = bi;
        ls[wave] = sm;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < 4; ++w) {
            band_best(b, bi, lb[w], li[w]);
            sm = fmax(sm, ls[w]);
        }
        pb[blockIdx.x] = b;
        pi[blockIdx.x] = bi;
        ps[blockIdx.x] = sm;
    }
}

// Reduce the scan's nb partials and decide the step (phase 0, 1, 2 as above);
// a pick covers its rows.  One workgroup of 1024 threads.
__global__ __launch_bounds__(1024) void k_band_decide(int phase, int step, int nb, const double *__restrict__ pb,
                                                      const int *__restrict__ pi, const double *__restrict__ ps,
                                                      BandState *st, int *done, const int64_t *__restrict__ off,
                                                      const int *__restrict__ len, const int *__restrict__ row,
                                                      const float *__restrict__ val, float *cur, uint8_t *picked,
                                                      int *picks, double *pgain) {
    __shared__ double lb[16], ls[16];
    __shared__ int li[16];
    __shared__ int top;
    if (*done || st->decided == step) return;
    double b = -1.0, sm = -1.0;
    int bi = -1;
    if (static_cast<int>(threadIdx.x) < nb) {
        b = pb[threadIdx.x];
        bi = pi[threadIdx.x];
        sm = ps[threadIdx.x];
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const double ob = __shfl_xor(b, o, 64);
        const int oi = __shfl_xor(bi, o, 64);
        band_best(b, bi, ob, oi);
        sm = fmax(sm, __shfl_xor(sm, o, 64));
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) {
        lb[wave] = b;
        li[wave] = bi;
        ls[wave] = sm;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < 16; ++w) {
            band_best(b, bi, lb[w], li[w]);
            sm = fmax(sm, ls[w]);
        }
        int pick = -1;
        if (bi >= 0 && b > 0.0 && b > sm) {
            pick = bi;
            picked[bi] = 1;
            picks[step] = bi;
            pgain[step] = b;
            st->decided = step;
        } else if (phase == 2 || (phase == 0 && !(sm > 0.0))) {
            *done = 1;       // no positive increment is left
        } else {
            st->thr = phase == 0 ? sm : (bi >= 0 && b > 0.0 ? b : 0.0);
        }
        top = pick;
    }
    __syncthreads();
    const int c = top;
    if (c < 0) return;
    // the range's live entries hold distinct rows (at most one entry per row
    // and candidate); a compacted range may repeat a row at a position filled
    // with Lbar = -inf, which never raises a cover and so never writes
    for (int64_t e = off[c] + threadIdx.x; e < off[c] + len[c]; e += 1024) {
        const int r = row[e];
        const float v = val[e];
        if (v > cur[r]) cur[r] = v;
    }
}

__global__ void k_len_init(const int64_t *__restrict__ off, int n, int *__restrict__ len) {
    for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < n; c += gridDim.x * blockDim.x)
        len[c] = static_cast<int>(off[c + 1] - off[c]);
}

// Recompute every stale bound at or above the threshold (and positive), one
// wave per such candidate with k_gain's summation order.  len[c]: the
// candidate's current range [off[c], off[c] + len[c]).  With compact the
// range is compacted on the way (lane_gain_compact): the new length ends at
// the last kept entry, and positions below it that no lane keeps are filled
// with Lbar = -inf (never above a cover, adding exactly 0).
__global__ __launch_bounds__(64) void k_band_refresh(const int64_t *__restrict__ off, int *row, float *val,
                                                     const float *__restrict__ cur,
                                                     const uint8_t *__restrict__ picked, double *ub, int *stamp,
                                                     int *len, int compact, int n, int step,
                                                     const BandState *__restrict__ st,
                                                     const int *__restrict__ done) {
    if (*done || st->decided == step) return;
    const double thr = st->thr;
    const int lane = threadIdx.x;
    for (int c0 = blockIdx.x * 64; c0 < n; c0 += gridDim.x * 64) {
        const int c = c0 + lane;
        bool q = false;
        if (c < n && !picked[c] && stamp[c] != step) {
            const double g = ub[c];
            q = g > 0.0 && g >= thr;
        }
        unsigned long long m = __ballot(q);
        while (m) {
            const int cc = c0 + __builtin_ctzll(m);
            m &= m - 1;
            const int64_t e0 = off[cc];
            const int L = len[cc];
            double s;
            if (compact) {
                int nl;
                s = wave_sum(lane_gain_compact(e0, L, lane, row, val, cur, nl));
                int last = nl > 0 ? 64 * (nl - 1) + lane + 1 : 0;
#pragma unroll
                for (int o = 32; o > 0; o >>= 1) last = max(last, __shfl_xor(last, o, 64));
                for (int64_t p = e0 + lane + 64 * static_cast<int64_t>(nl); p < e0 + last; p += 64)
                    val[p] = -INFINITY;
                if (lane == 0) len[cc] = last;
            } else {
                s = wave_sum(lane_gain(e0, e0 + L, lane, row, val, cur));
            }
            if (lane == 0) {
                ub[cc] = s;
                stamp[cc] = step;
            }
        }
    }
}

__global__ void k_set_i64(int64_t *p, int64_t v) { *p = v; }
// Same-block (detected, model) pairs of one batch, added to *acc: over the
// (block, candidate) slots, model spots of the slot times detected spots of
// its block; keep (may be NULL) limits the sum to kept candidates.
__global__ __launch_bounds__(256) void k_slot_pairs(const int64_t *__restrict__ offs,
                                                    const int64_t *__restrict__ ooff, int nb, int C,
                                                    const uint8_t *__restrict__ keep,
                                                    unsigned long long *__restrict__ acc) {
    unsigned long long t = 0;
    const int64_t L = static_cast<int64_t>(nb) * C;
    for (int64_t k = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; k < L;
         k += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        const int b = static_cast<int>(k / C), c = static_cast<int>(k - static_cast<int64_t>(b) * C);
        if (keep && !keep[c]) continue;
        t += static_cast<unsigned long long>((offs[k + 1] - offs[k]) * (ooff[b + 1] - ooff[b]));
    }
    for (int o = 32; o > 0; o >>= 1) t += __shfl_xor(t, o);
    if ((threadIdx.x & 63) == 0 && t) atomicAdd(acc, t);
}
__global__ void k_fill_f(float *p, int64_t n, float v) {
    int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}
__global__ void k_fill_u8(uint8_t *p, int64_t n, uint8_t v) {
    int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}
__global__ void k_fill_i(int *p, int64_t n, int v) {
    int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

}  // namespace laue

using namespace laue;

// ---------------------------------------------------------------- host: candidates

namespace {

struct CandWs {
    PairTab *tab;
    double *angw;
    float *nrat;
    int64_t *ooff;
    int *counts;
    int64_t *offs;
};

size_t carve_cand(Carver &cv, CandWs &w, int M, int nb, int64_t n_pairs) {
    w.tab = cv.take<PairTab>(1);
    w.angw = cv.take<double>(static_cast<size_t>(kMaxReps) * std::max(M, 1));
    w.nrat = cv.take<float>(std::max(M, 1));
    w.ooff = cv.take<int64_t>(nb + 1);
    w.counts = cv.take<int>(std::max<int64_t>(n_pairs, 1));
    w.offs = cv.take<int64_t>(std::max<int64_t>(n_pairs, 1) + 1);
    return cv.size();
}

int validate_obs_host(const laue_obs_spots *o, int nb) {
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

}  // namespace

extern "C" size_t laue_candidates_workspace_size(const laue_geometry *geom, int32_t n_planes,
                                                 int64_t n_pairs) {
    if (!geom || validate_geometry(geom) != LAUE_OK || n_planes < 0 || n_pairs < 0) return 0;
    Carver cv(nullptr);
    CandWs w;
    return carve_cand(cv, w, n_planes, geom->n_rot * geom->n_det, n_pairs);
}

extern "C" int laue_candidates_generate(const laue_geometry *geom, const laue_planes *planes,
                                        const laue_obs_spots *obs, const laue_cand_params *par,
                                        laue_candidates *out, int64_t *n_found, void *ws,
                                        size_t ws_bytes, void *stream) {
    clear_error();
    int rc;
    if ((rc = validate_geometry(geom)) || (rc = validate_planes(planes))) return rc;
    const int nb = geom->n_rot * geom->n_det;
    if ((rc = validate_obs_host(obs, nb))) return rc;
    LAUE_REQUIRE(par && out && n_found && out->q, LAUE_EINVAL, "NULL argument");
    LAUE_REQUIRE(par->n_pairs >= 0 && par->n_pairs < (int64_t(1) << 31), LAUE_EINVAL, "bad n_pairs");
    LAUE_REQUIRE((par->pair_a == nullptr) == (par->pair_b == nullptr), LAUE_EINVAL,
                 "pair_a and pair_b must both be given or both be NULL");
    LAUE_REQUIRE(std::isfinite(par->delta_deg) && par->delta_deg > 0 && par->delta_deg < 90,
                 LAUE_EINVAL, "bad angle tolerance");
    hipStream_t s = static_cast<hipStream_t>(stream);
    Carver cv(ws);
    CandWs w;
    size_t need = carve_cand(cv, w, planes->n, nb, par->n_pairs);
    if ((rc = check_ws(ws, ws_bytes, need))) return rc;
    // plane tables on the host: family representatives (w_x >= w_y >= w_z >= 0),
    // pairwise angles in FP64 (NaN for parallel planes), N / N_max from d
    const int M = planes->n;
    std::vector<float> hw(3 * M), hd(M);
    LAUE_CHECK_HIP(hipMemcpyAsync(hw.data(), planes->w, 3 * M * sizeof(float), hipMemcpyDeviceToHost, s));
    LAUE_CHECK_HIP(hipMemcpyAsync(hd.data(), planes->d, M * sizeof(float), hipMemcpyDeviceToHost, s));
    LAUE_CHECK_HIP(hipStreamSynchronize(s));
    // one representative per orbit of the 24 proper cubic rotations (signed
    // permutation matrices of determinant +1; exact on FP32 normals), the first
    // plane of each orbit in list order
    PairTab tab{};
    tab.M = M;
    {
        std::vector<char> covered(M, 0);
        const int perms[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};
        const int psign[6] = {1, -1, -1, 1, 1, -1};
        for (int m = 0; m < M; ++m) {
            if (covered[m]) continue;
            LAUE_REQUIRE(tab.n_rep < kMaxReps, LAUE_EINVAL, "too many plane families");
            tab.rep[tab.n_rep++] = m;
            for (int pi = 0; pi < 6; ++pi)
                for (int sg = 0; sg < 8; ++sg) {
                    const int s0 = (sg & 1) ? -1 : 1, s1 = (sg & 2) ? -1 : 1, s2 = (sg & 4) ? -1 : 1;
                    if (psign[pi] * s0 * s1 * s2 != 1) continue;
                    const float v[3] = {s0 * hw[3 * m + perms[pi][0]], s1 * hw[3 * m + perms[pi][1]],
                                        s2 * hw[3 * m + perms[pi][2]]};
                    // same normal and same spacing (harmonics share the normal)
                    for (int j = 0; j < M; ++j)
                        if (hd[j] == hd[m] && hw[3 * j] == v[0] && hw[3 * j + 1] == v[1] &&
                            hw[3 * j + 2] == v[2]) {
                            covered[j] = 1;
                            break;
                        }
                }
        }
    }
    std::vector<double> angw(static_cast<size_t>(tab.n_rep) * M);
    for (int r = 0; r < tab.n_rep; ++r) {
        const int a = tab.rep[r];
        for (int m = 0; m < M; ++m) {
            double c = 0.0;
            for (int k = 0; k < 3; ++k) c += static_cast<double>(hw[3 * a + k]) * hw[3 * m + k];
            const bool par_ = std::fabs(std::fabs(c) - 1.0) < 1e-6;
            angw[static_cast<size_t>(r) * M + m] = par_ ? std::nan("") : std::acos(std::max(-1.0, std::min(1.0, c)));
        }
    }
    float dmin = *std::min_element(hd.begin(), hd.end());
    std::vector<float> nrat(M);
    for (int m = 0; m < M; ++m) nrat[m] = static_cast<float>((static_cast<double>(dmin) * dmin) / (static_cast<double>(hd[m]) * hd[m]));
    LAUE_CHECK_HIP(hipMemcpyAsync(w.tab, &tab, sizeof(PairTab), hipMemcpyHostToDevice, s));
    LAUE_CHECK_HIP(hipMemcpyAsync(w.angw, angw.data(), angw.size() * sizeof(double), hipMemcpyHostToDevice, s));
    LAUE_CHECK_HIP(hipMemcpyAsync(w.nrat, nrat.data(), M * sizeof(float), hipMemcpyHostToDevice, s));
    LAUE_CHECK_HIP(hipMemcpyAsync(w.ooff, obs->block_off, (nb + 1) * sizeof(int64_t), hipMemcpyHostToDevice, s));
    const uint32_t k0 = static_cast<uint32_t>(par->seed & 0xffffffffu), k1 = static_cast<uint32_t>(par->seed >> 32);
    const double delta = par->delta_deg * M_PI / 180.0;
    const double l_side = 2.0 * geom->det[0].half_size;
    const int64_t P = par->n_pairs;
    int64_t total = 0;
    if (P > 0) {
        const unsigned nbk = static_cast<unsigned>((P + 127) / 128);
        k_pairs<<<nbk, 128, 0, s>>>(0, *geom, obs->p1, obs->p2, w.ooff, planes->w, planes->d, w.tab,
                                     w.angw, w.nrat, P, k0, k1, delta, l_side, w.counts, nullptr, 0,
                                     nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, par->pair_a,
                                     par->pair_b);
        LAUE_CHECK_HIP(hipGetLastError());
        if ((rc = launch_scan(w.counts, w.offs, P, s))) return rc;
        LAUE_CHECK_HIP(hipMemcpyAsync(&total, w.offs + P, sizeof(int64_t), hipMemcpyDeviceToHost, s));
        LAUE_CHECK_HIP(hipStreamSynchronize(s));
    }
    *n_found = total;
    const int64_t cap = out->n;
    if (total > 0 && cap > 0) {
        k_pairs<<<static_cast<unsigned>((P + 127) / 128), 128, 0, s>>>(
            1, *geom, obs->p1, obs->p2, w.ooff, planes->w, planes->d, w.tab, w.angw, w.nrat, P, k0, k1,
            delta, l_side, nullptr, w.offs, cap, out->q, out->pair, out->ma, out->mb, out->spot_a,
            out->spot_b, out->feat, par->pair_a, par->pair_b);
        LAUE_CHECK_HIP(hipGetLastError());
    }
    out->n = std::min(total, cap);
    LAUE_CHECK_HIP(hipStreamSynchronize(s));
    return LAUE_OK;
}

// ---------------------------------------------------------------- cell index

namespace laue {

// Per block: the bounding box of its detected spots and the grid's cell size.
__global__ __launch_bounds__(256) void k_cell_box(const float *__restrict__ P1, const float *__restrict__ P2,
                                                  const int64_t *__restrict__ ooff, float4 *__restrict__ box) {
    const int b = blockIdx.x;
    const int64_t r0 = ooff[b], r1 = ooff[b + 1];
    float x0 = INFINITY, x1 = -INFINITY, y0 = INFINITY, y1 = -INFINITY;
    for (int64_t i = r0 + threadIdx.x; i < r1; i += blockDim.x) {
        const float u = P1[i], v = P2[i];
        x0 = fminf(x0, u);
        x1 = fmaxf(x1, u);
        y0 = fminf(y0, v);
        y1 = fmaxf(y1, v);
    }
    __shared__ float red[4][256];
    red[0][threadIdx.x] = x0;
    red[1][threadIdx.x] = -x1;
    red[2][threadIdx.x] = y0;
    red[3][threadIdx.x] = -y1;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (static_cast<int>(threadIdx.x) < o)
            for (int q = 0; q < 4; ++q) red[q][threadIdx.x] = fminf(red[q][threadIdx.x], red[q][threadIdx.x + o]);
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        x0 = red[0][0];
        x1 = -red[1][0];
        y0 = red[2][0];
        y1 = -red[3][0];
        if (!(x0 <= x1)) x0 = x1 = 0.0f;
        if (!(y0 <= y1)) y0 = y1 = 0.0f;
        box[b] = make_float4(x0, y0, fmaxf((x1 - x0) / kCellG, 1e-6f), fmaxf((y1 - y0) / kCellG, 1e-6f));
    }
}

// Sort key of every detected spot: block * G^2 + cell (row-major cells of
// the G x G grid over the block's box; the box's cells are kCellG a side).
template <int G>
__global__ void k_cell_keys(const float *__restrict__ P1, const float *__restrict__ P2,
                            const int64_t *__restrict__ ooff, int nb, const float4 *__restrict__ box, int64_t n,
                            unsigned *__restrict__ key, int *__restrict__ idx) {
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
         i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        int lo = 0, hi = nb - 1;            // the block b with ooff[b] <= i < ooff[b + 1]
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (ooff[mid] <= i) lo = mid;
            else hi = mid - 1;
        }
        const float4 bc = box[lo];
        const float cx = bc.z * (static_cast<float>(kCellG) / G), cy = bc.w * (static_cast<float>(kCellG) / G);
        const int ix = cell_coord<G>((P1[i] - bc.x) / cx), iy = cell_coord<G>((P2[i] - bc.y) / cy);
        key[i] = static_cast<unsigned>(lo) * (G * G) + static_cast<unsigned>(iy * G + ix);
        idx[i] = static_cast<int>(i);
    }
}

__global__ void k_cell_gather(const float *__restrict__ P1, const float *__restrict__ P2,
                              const int *__restrict__ idx, int64_t n, float *__restrict__ P1s,
                              float *__restrict__ P2s, float2 *__restrict__ P12s) {
    for (int64_t k = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; k < n;
         k += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        const int i = idx[k];
        P1s[k] = P1[i];
        P2s[k] = P2[i];
        P12s[k] = make_float2(P1[i], P2[i]);
    }
}

__global__ void k_cell_gather2(const float *__restrict__ P1, const float *__restrict__ P2,
                               const int *__restrict__ idx, int64_t n, float2 *__restrict__ P12) {
    for (int64_t k = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; k < n;
         k += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        const int i = idx[k];
        P12[k] = make_float2(P1[i], P2[i]);
    }
}

// cell_off[t] = first position whose key is >= t, t = 0 .. n_keys.
__global__ void k_cell_off(const unsigned *__restrict__ key, int64_t n, int64_t n_keys, int *__restrict__ off) {
    for (int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; t <= n_keys;
         t += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        int64_t lo = 0, hi = n;
        while (lo < hi) {
            const int64_t mid = (lo + hi) >> 1;
            if (static_cast<int64_t>(key[mid]) < t) lo = mid + 1;
            else hi = mid;
        }
        off[t] = static_cast<int>(lo);
    }
}

}  // namespace laue

// ---------------------------------------------------------------- host: scoring

namespace {

struct CellWs {
    unsigned *key_in, *key_out;
    int *idx_in, *idx_out;
    float *P1s, *P2s;
    float2 *P12s;
    float2 *P12f;    // fine grid order
    int *off;
    int *off_f;
    float4 *box;
    void *tmp;
    size_t tmp_bytes;
};

void carve_cells(Carver &cv, CellWs &w, int nb, int64_t n_obs) {
    const int64_t n = std::max<int64_t>(n_obs, 1);
    w.key_in = cv.take<unsigned>(n);
    w.key_out = cv.take<unsigned>(n);
    w.idx_in = cv.take<int>(n);
    w.idx_out = cv.take<int>(n);
    w.P1s = cv.take<float>(n);
    w.P2s = cv.take<float>(n);
    w.P12s = cv.take<float2>(n);
    w.P12f = cv.take<float2>(n);
    w.off = cv.take<int>(static_cast<int64_t>(nb) * kCells + 1);
    w.off_f = cv.take<int>(static_cast<int64_t>(nb) * kFineCells + 1);
    w.box = cv.take<float4>(nb);
    size_t tmp = 0;
    (void)hipcub::DeviceRadixSort::SortPairs(nullptr, tmp, static_cast<unsigned *>(nullptr),
                                             static_cast<unsigned *>(nullptr), static_cast<int *>(nullptr),
                                             static_cast<int *>(nullptr), static_cast<int>(n));
    w.tmp_bytes = tmp;
    w.tmp = cv.take<char>(tmp);
}

// The cell index of the detected spots (stable: spots of one cell keep their order).
int build_cells(CellWs &w, const laue_obs_spots *obs, const int64_t *ooff_dev, int nb, hipStream_t s) {
    const int64_t n = obs->n;
    k_cell_box<<<nb, 256, 0, s>>>(obs->p1, obs->p2, ooff_dev, w.box);
    LAUE_CHECK_HIP(hipGetLastError());
    // the kCellG grid (per-(block, candidate) passes), then the kFineG grid
    // (per-model-spot pass); both sorts are stable
    for (int fine = 0; fine < 2; ++fine) {
        const int64_t n_keys = static_cast<int64_t>(nb) * (fine ? kFineCells : kCells);
        if (n > 0) {
            const unsigned g = static_cast<unsigned>(std::min<int64_t>((n + 255) / 256, 4096));
            if (fine)
                k_cell_keys<kFineG><<<g, 256, 0, s>>>(obs->p1, obs->p2, ooff_dev, nb, w.box, n, w.key_in, w.idx_in);
            else
                k_cell_keys<kCellG><<<g, 256, 0, s>>>(obs->p1, obs->p2, ooff_dev, nb, w.box, n, w.key_in, w.idx_in);
            LAUE_CHECK_HIP(hipGetLastError());
            int end_bit = 1;
            while (end_bit < 32 && (int64_t(1) << end_bit) <= n_keys) ++end_bit;
            size_t tb = w.tmp_bytes;
            LAUE_CHECK_HIP(hipcub::DeviceRadixSort::SortPairs(w.tmp, tb, w.key_in, w.key_out, w.idx_in, w.idx_out,
                                                             static_cast<int>(n), 0, end_bit, s));
            if (fine)
                k_cell_gather2<<<g, 256, 0, s>>>(obs->p1, obs->p2, w.idx_out, n, w.P12f);
            else
                k_cell_gather<<<g, 256, 0, s>>>(obs->p1, obs->p2, w.idx_out, n, w.P1s, w.P2s, w.P12s);
            LAUE_CHECK_HIP(hipGetLastError());
        }
        const unsigned go = static_cast<unsigned>(std::min<int64_t>((n_keys + 1 + 255) / 256, 4096));
        k_cell_off<<<go, 256, 0, s>>>(w.key_out, n, n_keys, fine ? w.off_f : w.off);
        LAUE_CHECK_HIP(hipGetLastError());
    }
    return LAUE_OK;
}

struct ScoreWs {
    EnumWs e;
    int *plane, *grain, *block;
    Col8 *colsE, *colsC;
    double *st;       // per model spot: the kStat statistics of the last pass
    double *hg;       // per candidate: its summed normal equations (kHg values)
    int *hcnt;        // per model spot: its SPOT entries (scoring passes)
    float *rad2;      // per model spot: squared zero radius (per-spot pass)
    unsigned long long *nbr;   // per model spot: slot spots whose zero disks meet its own
    int *unm, *lcnt;
    uint8_t *keep;
    int64_t *loff;
    int64_t *ooff;
    int *maxc;
    int64_t *pairs;   // pairs of all slots, of the kept candidates' slots, evaluated by the refinement,
                      // evaluated by the scoring
    CellWs cells;
};

size_t carve_score(Carver &cv, ScoreWs &w, const laue_geometry *g, int chunk, int64_t spot_cap, int64_t n_obs) {
    const int nb = g->n_rot * g->n_det;
    carve_enum(cv, w.e, g, chunk);
    carve_cells(cv, w.cells, nb, n_obs);
    const int64_t S = std::max<int64_t>(spot_cap, 1);
    w.plane = cv.take<int>(S);
    w.grain = cv.take<int>(S);
    w.block = cv.take<int>(S);
    w.colsE = cv.take<Col8>(S);
    w.colsC = cv.take<Col8>(S);
    w.st = cv.take<double>(static_cast<size_t>(S) * kStat);
    w.hg = cv.take<double>(static_cast<size_t>(std::max(chunk, 1)) * kHg);
    w.hcnt = cv.take<int>(S);
    w.rad2 = cv.take<float>(S);
    w.nbr = cv.take<unsigned long long>(S);
    w.unm = cv.take<int>(static_cast<size_t>(chunk) * nb);
    w.lcnt = cv.take<int>(static_cast<size_t>(chunk) * nb + 1);
    w.loff = cv.take<int64_t>(static_cast<size_t>(chunk) * nb + 1);
    w.keep = cv.take<uint8_t>(chunk);
    w.ooff = cv.take<int64_t>(nb + 1);
    w.maxc = cv.take<int>(1);
    w.pairs = cv.take<int64_t>(4);
    return cv.size();
}

// The statistics pass: per model spot at the E-step geometry (the first
// Gauss-Newton step), per (block, candidate) wave otherwise.
int launch_acc(const SlotArgs &A, float K, float bin_e, float T_skip, int64_t M, float *rad2,
               unsigned long long *nbr, double *st, hipStream_t s) {
    if (A.colsC == A.colsE) {
        if (M > 0) {
            const unsigned g = static_cast<unsigned>(std::min<int64_t>((M + 255) / 256, 16384));
            k_spot_rad<<<g, 256, 0, s>>>(A.colsE, M, K, T_skip, rad2);
            k_spot_nbr<<<g, 256, 0, s>>>(A, rad2, M, nbr);
            k_spot_acc<<<static_cast<unsigned>((M + 255) / 256), 256, 0, s>>>(A, K, bin_e, rad2, nbr, M, st);
        }
    } else {
        k_single_acc<<<static_cast<unsigned>(A.nb) * A.C, 64, 0, s>>>(A, K, bin_e, T_skip, st);
    }
    LAUE_CHECK_HIP(hipGetLastError());
    return LAUE_OK;
}

// The scoring passes (k_spot_score); pass 0 also sets the scoring radii and
// disk masks that pass 1 reuses.
int launch_score(const SlotArgs &A, int pass, int64_t M, float twoD2, float K2, float floor_e, float c_out,
                 float Lhit, float *rad2, unsigned long long *nbr, int *hcnt, int *unm, int *lcnt,
                 const int64_t *loff, const uint8_t *keep, int *lrow, float *lval, unsigned long long *ev,
                 hipStream_t s) {
    const int64_t L = static_cast<int64_t>(A.nb) * A.C;
    if (pass == 0) {
        k_fill_int2<<<static_cast<unsigned>(std::min<int64_t>((L + 255) / 256, 4096)), 256, 0, s>>>(unm, lcnt, L);
        LAUE_CHECK_HIP(hipGetLastError());
    }
    if (M == 0) return LAUE_OK;
    const unsigned g = static_cast<unsigned>(std::min<int64_t>((M + 255) / 256, 16384));
    const unsigned gs = static_cast<unsigned>((M + 255) / 256);
    if (pass == 0) {
        SlotArgs B = A;
        B.colsE = A.colsC;      // the disks at the scoring geometry
        k_score_rad<<<g, 256, 0, s>>>(A, M, twoD2, K2, c_out, Lhit, rad2);
        k_spot_nbr<<<g, 256, 0, s>>>(B, rad2, M, nbr);
        k_spot_score<0><<<gs, 256, 0, s>>>(A, M, twoD2, K2, floor_e, c_out, rad2, nbr, hcnt, unm, lcnt, nullptr,
                                           nullptr, nullptr, nullptr, ev);
    } else {
        k_spot_score<1><<<gs, 256, 0, s>>>(A, M, twoD2, K2, floor_e, c_out, rad2, nbr, hcnt, nullptr, nullptr, loff,
                                           keep, lrow, lval, ev);
    }
    LAUE_CHECK_HIP(hipGetLastError());
    return LAUE_OK;
}

}  // namespace

extern "C" size_t laue_score_workspace_size(const laue_geometry *geom, int64_t n_obs,
                                            const laue_score_params *par) {
    if (!geom || !par || validate_geometry(geom) != LAUE_OK || par->chunk < 1 || par->max_spots_per_cand < 1 ||
        n_obs < 0 || n_obs >= (int64_t(1) << 31))
        return 0;
    Carver cv(nullptr);
    ScoreWs w;
    return carve_score(cv, w, geom, par->chunk, static_cast<int64_t>(par->chunk) * par->max_spots_per_cand, n_obs);
}

extern "C" int laue_score_candidates(const laue_geometry *geom, const laue_planes *planes,
                                     const laue_obs_spots *obs, laue_grains *cand,
                                     const laue_score_params *par, laue_score_out *out, void *ws,
                                     size_t ws_bytes, void *stream) {
    clear_error();
    int rc;
    if ((rc = validate_geometry(geom)) || (rc = validate_planes(planes)) || (rc = validate_grains(cand)))
        return rc;
    const int nb = geom->n_rot * geom->n_det;
    if ((rc = validate_obs_host(obs, nb))) return rc;
    LAUE_REQUIRE(par && out, LAUE_EINVAL, "NULL argument");
    LAUE_REQUIRE(par->chunk >= 1 && par->max_spots_per_cand >= 1 && par->k_refine >= 0 && par->k_gn >= 0,
                 LAUE_EINVAL, "bad scoring parameters");
    LAUE_REQUIRE(std::isfinite(par->sigma_mm) && par->sigma_mm > 0 && std::isfinite(par->distance) &&
                     par->distance > 0 && std::isfinite(par->c_out) && par->c_out > 0 &&
                     std::isfinite(par->f_out) && std::isfinite(par->mu_rel) && par->mu_rel >= 0 &&
                     std::isfinite(par->eps_start) && std::isfinite(par->eps_end) &&
                     par->eps_start > 0 && par->eps_end > 0 && std::isfinite(par->eps_cool) &&
                     par->eps_cool >= 0 && par->eps_cool <= 1 && std::isfinite(par->drop_log2) &&
                     par->drop_log2 >= 0,
                 LAUE_EINVAL, "bad scoring parameters");
    LAUE_REQUIRE(out->lbar_off && (out->lbar_cap == 0 || (out->lbar_row && out->lbar_val)), LAUE_EINVAL,
                 "SPOT output arrays are NULL");
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int chunk = par->chunk;
    const int64_t spot_cap = static_cast<int64_t>(chunk) * par->max_spots_per_cand;
    LAUE_REQUIRE(obs->n < (int64_t(1) << 31), LAUE_EINVAL, "scoring takes fewer than 2^31 detected spots");
    Carver cv(ws);
    ScoreWs w;
    size_t need = carve_score(cv, w, geom, chunk, spot_cap, obs->n);
    if ((rc = check_ws(ws, ws_bytes, need))) return rc;
    LAUE_CHECK_HIP(hipMemcpyAsync(w.ooff, obs->block_off, (nb + 1) * sizeof(int64_t), hipMemcpyHostToDevice, s));
    if ((rc = build_cells(w.cells, obs, w.ooff, nb, s))) return rc;
    const double l2e = 1.4426950408889634;
    const double D2 = par->distance * par->distance;
    const float twoD2 = static_cast<float>(2.0 * D2);
    const float K2 = static_cast<float>(2.0 * D2 * l2e / (2.0 * par->sigma_mm * par->sigma_mm));
    const float floor_e = static_cast<float>(std::exp(-par->c_out / (2.0 * par->sigma_mm * par->sigma_mm)));
    const float Lhit = static_cast<float>(par->c_out * l2e / (2.0 * par->sigma_mm * par->sigma_mm));
    int64_t lbar_total = 0;
    const int N = cand->n;
    out->pairs_streamed = 0;
    k_set_i64<<<1, 1, 0, s>>>(w.pairs, 0);
    k_set_i64<<<1, 1, 0, s>>>(w.pairs + 1, 0);
    k_set_i64<<<1, 1, 0, s>>>(w.pairs + 2, 0);
    k_set_i64<<<1, 1, 0, s>>>(w.pairs + 3, 0);
    LAUE_CHECK_HIP(hipGetLastError());
    unsigned long long *pairs = reinterpret_cast<unsigned long long *>(w.pairs);
    if (N == 0) {
        k_set_i64<<<1, 1, 0, s>>>(out->lbar_off, 0);
        LAUE_CHECK_HIP(hipGetLastError());
    }
    int logged = 0;
    for (int c0 = 0; c0 < N; c0 += chunk) {
        const int C = std::min(chunk, N - c0);
        if (log_enabled() && c0 >= static_cast<int64_t>(N) * logged / 10) {
            LAUE_CHECK_HIP(hipStreamSynchronize(s));
            log_line("score: %d of %d candidates, %lld SPOT entries", c0, N, static_cast<long long>(lbar_total));
            ++logged;
        }
        laue_grains sub{C, cand->q + 4 * static_cast<int64_t>(c0), cand->x + 3 * static_cast<int64_t>(c0)};
        std::vector<int64_t> hb;
        int64_t total = 0;
        if ((rc = enumerate_count(geom, planes, &sub, 1, w.e, hb, &total, s))) return rc;
        if (total > spot_cap) {
            set_error("candidate model spots " + std::to_string(total) + " exceed the batch capacity " +
                      std::to_string(spot_cap) + " (raise max_spots_per_cand or lower chunk)");
            return LAUE_ECAPACITY;
        }
        const int64_t L = static_cast<int64_t>(nb) * C;
        k_max_int<<<1, 256, 0, s>>>(w.e.counts, L, w.maxc);
        int maxc = 0;
        LAUE_CHECK_HIP(hipMemcpyAsync(&maxc, w.maxc, sizeof(int), hipMemcpyDeviceToHost, s));
        LAUE_CHECK_HIP(hipStreamSynchronize(s));
        LAUE_REQUIRE(maxc <= 64, LAUE_ECAPACITY, "a candidate has more than 64 model spots in one block");
        if ((rc = launch_enumerate_ids(geom, planes, w.e, C, 1, total, w.plane, w.grain, w.block, s))) return rc;
        SlotArgs A;
        A.C = C;
        A.nb = nb;
        A.offs = w.e.offs;
        A.P1 = obs->p1;
        A.P2 = obs->p2;
        A.ooff = w.ooff;
        A.colsE = w.colsE;
        A.colsC = w.colsC;
        A.geom = w.e.geom;
        A.W = planes->w;
        A.n_planes = planes->n;
        A.grains = w.e.grains;
        A.mplane = w.plane;
        A.mgrain = w.grain;
        A.mblock = w.block;
        A.P1s = w.cells.P1s;
        A.P2s = w.cells.P2s;
        A.P12s = w.cells.P12s;
        A.P12f = w.cells.P12f;
        A.rowid_f = w.cells.idx_out;
        A.cell_off_f = w.cells.off_f;
        A.cell_off = w.cells.off;
        A.cbox = w.cells.box;
        A.evaluated = pairs + 2;
        // pairs of one pass over every slot (the refinement's k_refine * k_gn
        // statistics passes and the first scoring pass stream them all; the
        // second scoring pass streams the kept candidates' slots only)
        const unsigned pg = static_cast<unsigned>(std::min<int64_t>((L + 255) / 256, 1024));
        k_slot_pairs<<<pg, 256, 0, s>>>(w.e.offs, w.ooff, nb, C, nullptr, pairs);
        LAUE_CHECK_HIP(hipGetLastError());
        double eps_cooled = par->eps_start;
        for (int it = 0; it < par->k_refine; ++it) {
            const double eps = par->eps_cool > 0.0 ? eps_cooled
                               : par->k_refine == 1 ? par->eps_start
                               : par->eps_start * std::pow(par->eps_end / par->eps_start,
                                                           static_cast<double>(it) / (par->k_refine - 1));
            eps_cooled *= par->eps_cool;
            const float K = static_cast<float>(2.0 * D2 * l2e / eps);
            const float bin_e = static_cast<float>(std::exp(-par->c_out / eps));
            // skip threshold: terms below 2^-drop_log2 of the bin's (whose
            // exponent is c_out / (eps ln 2)), at most the FP32-zero exponent
            const float T_skip = par->drop_log2 > 0.0
                                     ? static_cast<float>(std::min<double>(kZeroExp2, par->drop_log2 +
                                                                                       par->c_out * l2e / eps))
                                     : kZeroExp2;
            if ((rc = launch_eval(w.e.geom, planes, w.e.grains, C, w.plane, w.grain, w.block, total,
                                  nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, w.colsE, s)))
                return rc;
            for (int k = 0; k < par->k_gn; ++k) {
                A.colsC = w.colsE;
                if (k > 0) {
                    if ((rc = launch_eval(w.e.geom, planes, w.e.grains, C, w.plane, w.grain, w.block,
                                          total, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr,
                                          w.colsC, s)))
                        return rc;
                    A.colsC = w.colsC;
                }
                if ((rc = launch_acc(A, K, bin_e, T_skip, total, w.rad2, w.nbr, w.st, s))) return rc;
                k_single_normal<<<C, 64, 0, s>>>(A, w.st, D2, w.hg);
                k_single_step<<<(C + 63) / 64, 64, 0, s>>>(C, w.hg, par->mu_rel, sub.q, sub.x, w.e.grains);
                LAUE_CHECK_HIP(hipGetLastError());
            }
        }
        // scoring at the refined grains
        if ((rc = launch_eval(w.e.geom, planes, w.e.grains, C, w.plane, w.grain, w.block, total,
                              nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, w.colsC, s)))
            return rc;
        A.colsC = w.colsC;
        if ((rc = launch_score(A, 0, total, twoD2, K2, floor_e, static_cast<float>(par->c_out), Lhit, w.rad2,
                               w.nbr, w.hcnt, w.unm, w.lcnt, nullptr, nullptr, nullptr, nullptr, pairs + 3, s)))
            return rc;
        k_single_keep<<<(C + 127) / 128, 128, 0, s>>>(C, nb, w.e.offs, w.unm, w.lcnt, par->f_out,
                                                      w.keep,
                                                      out->n_model ? out->n_model + c0 : nullptr,
                                                      out->n_unmatched ? out->n_unmatched + c0 : nullptr,
                                                      out->keep ? out->keep + c0 : nullptr);
        LAUE_CHECK_HIP(hipGetLastError());
        if ((rc = launch_scan(w.lcnt, w.loff, L, s))) return rc;
        int64_t ctot = 0;
        LAUE_CHECK_HIP(hipMemcpyAsync(&ctot, w.loff + L, sizeof(int64_t), hipMemcpyDeviceToHost, s));
        LAUE_CHECK_HIP(hipStreamSynchronize(s));
        if (lbar_total + ctot > out->lbar_cap) {
            out->lbar_n = lbar_total + ctot;
            set_error("SPOT entry capacity " + std::to_string(out->lbar_cap) + " exceeded");
            return LAUE_ECAPACITY;
        }
        k_cand_off<<<(C + 1 + 127) / 128, 128, 0, s>>>(w.loff, C, nb, lbar_total, out->lbar_off, c0, 1);
        LAUE_CHECK_HIP(hipGetLastError());
        if (ctot > 0) {
            k_slot_pairs<<<pg, 256, 0, s>>>(w.e.offs, w.ooff, nb, C, w.keep, pairs + 1);
            LAUE_CHECK_HIP(hipGetLastError());
        }
        if (ctot > 0 &&
            (rc = launch_score(A, 1, total, twoD2, K2, floor_e, static_cast<float>(par->c_out), Lhit, w.rad2,
                               w.nbr, w.hcnt, nullptr, nullptr, w.loff, w.keep, out->lbar_row + lbar_total,
                               out->lbar_val + lbar_total, pairs + 3, s)))
            return rc;
        lbar_total += ctot;
    }
    out->lbar_n = lbar_total;
    int64_t hp[4] = {0, 0, 0, 0};
    LAUE_CHECK_HIP(hipMemcpyAsync(hp, w.pairs, 4 * sizeof(int64_t), hipMemcpyDeviceToHost, s));
    LAUE_CHECK_HIP(hipStreamSynchronize(s));
    out->pairs_streamed = (static_cast<int64_t>(par->k_refine) * par->k_gn + 1) * hp[0] + hp[1];
    out->pairs_evaluated = hp[2] + hp[3];
    out->pairs_refine = static_cast<int64_t>(par->k_refine) * par->k_gn * hp[0];
    return LAUE_OK;
}

// ---------------------------------------------------------------- host: greedy

namespace {
struct GreedyWs {
    float *cur;
    uint8_t *picked;
    double *gain;   // upper bounds of the increments (exact at their stamp)
    int *stamp;
    int *len;       // current length of each candidate's range (compaction)
    int *done;
    double *pb, *ps;   // the band scan's per-block partials
    int *pi;
    BandState *st;
};

size_t carve_greedy(Carver &cv, GreedyWs &w, int n_cand, int64_t n_rows) {
    w.cur = cv.take<float>(std::max<int64_t>(n_rows, 1));
    w.picked = cv.take<uint8_t>(std::max(n_cand, 1));
    w.gain = cv.take<double>(std::max(n_cand, 1));
    w.stamp = cv.take<int>(std::max(n_cand, 1));
    w.len = cv.take<int>(std::max(n_cand, 1));
    w.done = cv.take<int>(1);
    w.pb = cv.take<double>(kBandScanBlocks);
    w.ps = cv.take<double>(kBandScanBlocks);
    w.pi = cv.take<int>(kBandScanBlocks);
    w.st = cv.take<BandState>(1);
    return cv.size();
}

// The selection on a SPOT matrix whose entries it may reorder within each
// candidate's range when compact (row and val then hold each range's live
// entries first; lbar_off is unchanged).
int greedy_run(const int64_t *lbar_off, int32_t *lbar_row, float *lbar_val, bool compact, int32_t n_cand,
               int64_t n_rows, double phi, int32_t k_max, int32_t *picks, double *gains, int32_t *n_picked,
               GreedyWs &w, hipStream_t s) {
    *n_picked = 0;
    if (n_cand == 0 || k_max == 0) return LAUE_OK;
    k_fill_f<<<static_cast<unsigned>((std::max<int64_t>(n_rows, 1) + 255) / 256), 256, 0, s>>>(w.cur, n_rows, static_cast<float>(phi));
    k_fill_u8<<<(n_cand + 255) / 256, 256, 0, s>>>(w.picked, n_cand, 0);
    k_fill_i<<<1, 64, 0, s>>>(w.done, 1, 0);
    k_fill_i<<<(k_max + 255) / 256, 256, 0, s>>>(picks, k_max, -1);
    k_band_init<<<1, 1, 0, s>>>(w.st);
    k_len_init<<<static_cast<unsigned>(std::min((n_cand + 255) / 256, 4096)), 256, 0, s>>>(lbar_off, n_cand, w.len);
    LAUE_CHECK_HIP(hipGetLastError());
    const int K = std::min(k_max, n_cand);
    // every increment once: exact at step 0
    k_gain<<<n_cand, 64, 0, s>>>(lbar_off, lbar_row, lbar_val, w.cur, w.picked, w.gain, w.done, n_cand);
    k_fill_i<<<(n_cand + 255) / 256, 256, 0, s>>>(w.stamp, n_cand, 0);
    const int nb = std::min(kBandScanBlocks, (n_cand + 255) / 256);
    const int nr = std::min(kBandRefreshWaves, (n_cand + 63) / 64);
    for (int step = 0; step < K; ++step) {
        for (int phase = 0; phase < 3; ++phase) {
            if (phase > 0)
                k_band_refresh<<<nr, 64, 0, s>>>(lbar_off, lbar_row, lbar_val, w.cur, w.picked, w.gain, w.stamp,
                                                 w.len, compact ? 1 : 0, n_cand, step, w.st, w.done);
            k_band_scan<<<nb, 256, 0, s>>>(w.picked, w.gain, w.stamp, n_cand, step, w.st, w.done, w.pb, w.pi, w.ps);
            k_band_decide<<<1, 1024, 0, s>>>(phase, step, nb, w.pb, w.pi, w.ps, w.st, w.done, lbar_off, w.len,
                                             lbar_row, lbar_val, w.cur, w.picked, picks, gains);
        }
        LAUE_CHECK_HIP(hipGetLastError());
        if (step % 64 == 63 && step + 1 < K) {   // stop launching once the selection has ended
            int dn = 0;
            LAUE_CHECK_HIP(hipMemcpyAsync(&dn, w.done, sizeof(int), hipMemcpyDeviceToHost, s));
            LAUE_CHECK_HIP(hipStreamSynchronize(s));
            if (dn) break;
        }
    }
    std::vector<int> hp(K);
    LAUE_CHECK_HIP(hipMemcpyAsync(hp.data(), picks, K * sizeof(int), hipMemcpyDeviceToHost, s));
    LAUE_CHECK_HIP(hipStreamSynchronize(s));
    int n = 0;
    while (n < K && hp[n] >= 0) ++n;
    *n_picked = n;
    return LAUE_OK;
}
}  // namespace

extern "C" size_t laue_spot_greedy_workspace_size(int32_t n_cand, int64_t n_rows) {
    if (n_cand < 0 || n_rows < 0) return 0;
    Carver cv(nullptr);
    GreedyWs w;
    return carve_greedy(cv, w, n_cand, n_rows);
}

#define GREEDY_ARGS_OK()                                                                                  \
    LAUE_REQUIRE(n_cand >= 0 && n_rows >= 0 && k_max >= 0 && n_picked, LAUE_EINVAL, "bad sizes");       \
    LAUE_REQUIRE(n_cand == 0 || (lbar_off && lbar_row && lbar_val), LAUE_EINVAL, "SPOT arrays are NULL"); \
    LAUE_REQUIRE(k_max == 0 || (picks && gains), LAUE_EINVAL, "outputs are NULL");                       \
    LAUE_REQUIRE(std::isfinite(phi), LAUE_EINVAL, "phi must be finite")

extern "C" int laue_spot_greedy(const int64_t *lbar_off, const int32_t *lbar_row,
                                const float *lbar_val, int32_t n_cand, int64_t n_rows, double phi,
                                int32_t k_max, int32_t *picks, double *gains, int32_t *n_picked,
                                void *ws, size_t ws_bytes, void *stream) {
    clear_error();
    int rc;
    GREEDY_ARGS_OK();
    hipStream_t s = static_cast<hipStream_t>(stream);
    Carver cv(ws);
    GreedyWs w;
    const size_t need = carve_greedy(cv, w, n_cand, n_rows);
    if ((rc = check_ws(ws, ws_bytes, need))) return rc;
    *n_picked = 0;
    if (n_cand == 0 || k_max == 0) return LAUE_OK;
    // room for a copy of the entries: the selection compacts the copy
    int64_t n_ent = 0;
    LAUE_CHECK_HIP(hipMemcpyAsync(&n_ent, lbar_off + n_cand, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    LAUE_CHECK_HIP(hipStreamSynchronize(s));
    int64_t e_first = 0;
    LAUE_CHECK_HIP(hipMemcpyAsync(&e_first, lbar_off, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    LAUE_CHECK_HIP(hipStreamSynchronize(s));
    int32_t *row = const_cast<int32_t *>(lbar_row);
    float *val = const_cast<float *>(lbar_val);
    bool compact = false;
    if (e_first == 0 && n_ent > 0) {
        Carver cc(static_cast<char *>(ws) + need);
        int32_t *row_c = cc.take<int32_t>(n_ent);
        float *val_c = cc.take<float>(n_ent);
        if (need + cc.size() <= ws_bytes) {
            LAUE_CHECK_HIP(hipMemcpyAsync(row_c, lbar_row, n_ent * sizeof(int32_t), hipMemcpyDeviceToDevice, s));
            LAUE_CHECK_HIP(hipMemcpyAsync(val_c, lbar_val, n_ent * sizeof(float), hipMemcpyDeviceToDevice, s));
            row = row_c;
            val = val_c;
            compact = true;
        }
    }
    return greedy_run(lbar_off, row, val, compact, n_cand, n_rows, phi, k_max, picks, gains, n_picked, w, s);
}

namespace laue {
int spot_greedy_inplace(const int64_t *lbar_off, int32_t *lbar_row, float *lbar_val, int32_t n_cand,
                        int64_t n_rows, double phi, int32_t k_max, int32_t *picks, double *gains,
                        int32_t *n_picked, void *ws, size_t ws_bytes, void *stream) {
    clear_error();
    int rc;
    GREEDY_ARGS_OK();
    hipStream_t s = static_cast<hipStream_t>(stream);
    Carver cv(ws);
    GreedyWs w;
    const size_t need = carve_greedy(cv, w, n_cand, n_rows);
    if ((rc = check_ws(ws, ws_bytes, need))) return rc;
    return greedy_run(lbar_off, lbar_row, lbar_val, true, n_cand, n_rows, phi, k_max, picks, gains, n_picked, w, s);
}
}  // namespace laue
