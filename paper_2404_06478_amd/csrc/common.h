// Internal definitions shared by the HIP translation units of liblaueot.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/laueot.h"

namespace laue {

// ---------------------------------------------------------------- errors

void set_error(const std::string &msg);
void clear_error();
// progress lines on stderr when the environment sets LAUE_LOG (not "0")
bool log_enabled();
void log_line(const char *fmt, ...) __attribute__((format(printf, 1, 2)));

#define LAUE_CHECK_HIP(expr)                                                        \
    do {                                                                            \
        hipError_t _e = (expr);                                                     \
        if (_e != hipSuccess) {                                                     \
            ::laue::set_error(std::string("HIP error in ") + #expr + ": " +         \
                              hipGetErrorString(_e));                               \
            return LAUE_EDEVICE;                                                    \
        }                                                                           \
    } while (0)

#define LAUE_REQUIRE(cond, code, msg)                                               \
    do {                                                                            \
        if (!(cond)) {                                                              \
            ::laue::set_error(msg);                                                 \
            return (code);                                                          \
        }                                                                           \
    } while (0)

// ---------------------------------------------------------------- geometry

// Detector in FP32: centre, normal, in-plane axes, half side.
struct DetF {
    float c[3], n[3], a1[3], a2[3];
    float half;
};

// Device-resident copy of the scan geometry (read through scalar loads).
struct GeomF {
    int n_rot, n_det;
    float lam_min, lam_max;
    DetF det[LAUE_MAX_DET];
    float cs[LAUE_MAX_ROT][2];   // cos, sin of omega_t (rounded from FP64)
};

int validate_geometry(const laue_geometry *g);
void make_geomf(const laue_geometry *g, GeomF *out);

// Grain in FP32 for the forward model: R (row-major 3x3) and x.
struct GrainF {
    float R[9];
    float x[3];
};

// FP32 grain from an FP64 quaternion (normalised) and position.
__device__ inline GrainF grain_f32(const double *q, const double *x) {
    double w = q[0], a = q[1], b = q[2], c = q[3];
    const double nrm = sqrt(w * w + a * a + b * b + c * c);
    w /= nrm; a /= nrm; b /= nrm; c /= nrm;
    const double R[9] = {1 - 2 * (b * b + c * c), 2 * (a * b - w * c),     2 * (a * c + w * b),
                         2 * (a * b + w * c),     1 - 2 * (a * a + c * c), 2 * (b * c - w * a),
                         2 * (a * c - w * b),     2 * (b * c + w * a),     1 - 2 * (a * a + b * b)};
    GrainF g;
    for (int k = 0; k < 9; ++k) g.R[k] = static_cast<float>(R[k]);
    for (int k = 0; k < 3; ++k) g.x[k] = static_cast<float>(x[k]);
    return g;
}

// ---------------------------------------------------------------- workspace

// Bump allocator over a caller workspace; with base == nullptr it only sizes.
struct Carver {
    char *base;
    size_t off = 0;
    explicit Carver(void *b) : base(static_cast<char *>(b)) {}
    template <class T>
    T *take(size_t count) {
        off = (off + 255) & ~size_t(255);
        T *p = base ? reinterpret_cast<T *>(base + off) : nullptr;
        off += count * sizeof(T);
        return p;
    }
    size_t size() const { return (off + 255) & ~size_t(255); }
};

int check_ws(void *ws, size_t ws_bytes, size_t need);

// number of temperatures of an EM run (the stage schedule, or the cooling
// from eps_start down to eps_end), without the final iterations
int em_n_temperatures(const laue_em_params &p);

// laue_spot_greedy on a SPOT matrix the selection may reorder: each
// candidate's live entries are compacted to the front of its range as the
// selection goes (the picks and increments are those of laue_spot_greedy).
int spot_greedy_inplace(const int64_t *lbar_off, int32_t *lbar_row, float *lbar_val, int32_t n_cand,
                        int64_t n_rows, double phi, int32_t k_max, int32_t *picks, double *gains,
                        int32_t *n_picked, void *ws, size_t ws_bytes, void *stream);

// ---------------------------------------------------------------- device math

// Plane normal in the lab: u = Gamma_t R w (Sec. 3.3), explicit FMA chains.
__device__ __forceinline__ void lab_normal(const float *R, float c, float s, float wx, float wy,
                                           float wz, float &ux, float &uy, float &uz) {
    float vx = fmaf(R[2], wz, fmaf(R[1], wy, R[0] * wx));
    float vy = fmaf(R[5], wz, fmaf(R[4], wy, R[3] * wx));
    float vz = fmaf(R[8], wz, fmaf(R[7], wy, R[6] * wx));
    ux = fmaf(-s, vy, c * vx);
    uy = fmaf(s, vx, c * vy);
    uz = vz;
}

// Result of the forward model for one (plane, grain, rotation, detector).
struct SpotGeo {
    float lam;
    float s1, s2;          // detector-local position
    float vn, v1, v2;      // ray vector tau * r in the detector frame
    bool inband;
    bool on;               // tau > 0 and inside the detector square
    uint8_t flags;         // bit0 near band edge, bit1 near detector edge
};

// Forward model (Eqs. wavelength_lambda, ray_mnt, s_mnt, model_spot_cut) of
// plane (w, d) of grain (R, x) at rotation (c, s) on detector det.
__device__ __forceinline__ SpotGeo spot_geometry(const GeomF &G, const DetF &D, const float *R,
                                                 const float *x, float c, float s, float wx,
                                                 float wy, float wz, float dsp) {
    SpotGeo o;
    float ux, uy, uz;
    lab_normal(R, c, s, wx, wy, wz, ux, uy, uz);
    o.lam = 2.0f * dsp * ux;
    o.inband = (o.lam >= G.lam_min) && (o.lam <= G.lam_max);
    float rx = fmaf(-2.0f * ux, ux, 1.0f);
    float ry = -2.0f * ux * uy;
    float rz = -2.0f * ux * uz;
    float yx = fmaf(-s, x[1], c * x[0]);
    float yy = fmaf(s, x[0], c * x[1]);
    float yz = x[2];
    float den = fmaf(D.n[2], rz, fmaf(D.n[1], ry, D.n[0] * rx));
    float num = fmaf(D.n[2], D.c[2] - yz, fmaf(D.n[1], D.c[1] - yy, D.n[0] * (D.c[0] - yx)));
    float tau = num / den;
    float vx = tau * rx, vy = tau * ry, vz = tau * rz;
    float ex = yx + vx - D.c[0], ey = yy + vy - D.c[1], ez = yz + vz - D.c[2];
    o.s1 = fmaf(D.a1[2], ez, fmaf(D.a1[1], ey, D.a1[0] * ex));
    o.s2 = fmaf(D.a2[2], ez, fmaf(D.a2[1], ey, D.a2[0] * ex));
    o.vn = fmaf(D.n[2], vz, fmaf(D.n[1], vy, D.n[0] * vx));
    o.v1 = fmaf(D.a1[2], vz, fmaf(D.a1[1], vy, D.a1[0] * vx));
    o.v2 = fmaf(D.a2[2], vz, fmaf(D.a2[1], vy, D.a2[0] * vx));
    float inf = fmaxf(fabsf(o.s1), fabsf(o.s2));
    o.on = (tau > 0.0f) && (inf < D.half);
    uint8_t f = 0;
    if (fabsf(o.lam - G.lam_min) <= 1e-6f || fabsf(o.lam - G.lam_max) <= 1e-6f) f |= 1;
    if (fabsf(inf - D.half) <= 1e-4f) f |= 2;
    o.flags = f;
    return o;
}

// Packed column of the streamed cost (one model spot), 32 bytes:
// detector-local position, in-plane ray components, |v|^2, |v|^4 and the
// normal component of the ray vector v = tau r.
struct Col8 {
    float s1, s2, v1, v2, vv, vv2, vn, pad;
};

// Exponent (in log2 units) of one plan entry:  base - K * c'  with
// c = 2 D^2 c' the chord cost D^2 ||rhat - r||^2 (Sec. 4, L_ij up to a
// constant).  With v the model ray vector, delta = p - s the in-plane
// difference (exact when p and s are close) and d = v + delta:
//   c' = |v x d|^2 / (|v|^2 |d|^2 + (v.d) |v| |d|)
// which avoids the cancellation of 1 - rhat.r.  Since delta lies in the
// detector plane, |v x d|^2 = |v x delta|^2 = |v|^2 |delta|^2 - (v.delta)^2 and
// |v|^2 |d|^2 = |v|^4 + |v|^2 (2 v.delta + |delta|^2); neither cancels badly
// because the normal component of v is at least ~0.7 |v| on the detectors.
// 17 VALU + sqrt, rcp and exp per entry in the passes (a = |v|^2, a2 = |v|^4).
// c' = c / (2 D^2) of one (detected spot, model spot) pair.
__device__ __forceinline__ float chord_cp(float p1, float p2, float s1, float s2, float v1, float v2, float a,
                                          float a2) {
    const float dy = p1 - s1;
    const float dz = p2 - s2;
    const float e = fmaf(dz, dz, dy * dy);        // |delta|^2
    const float b = fmaf(v2, dz, v1 * dy);        // v.delta
    const float x2 = fmaf(a, e, -(b * b));        // |v x delta|^2
    const float vdd = a + b;                      // v.d
    const float w = fmaf(2.0f, b, e);             // |d|^2 - |v|^2
    const float P = fmaf(a, w, a2);               // |v|^2 |d|^2
    const float den = fmaf(vdd, __builtin_amdgcn_sqrtf(P), P);
    return x2 * __builtin_amdgcn_rcpf(den);
}

__device__ __forceinline__ float entry_exponent(float p1, float p2, float s1, float s2, float v1,
                                                float v2, float a, float a2, float K, float base) {
    return fmaf(-K, chord_cp(p1, p2, s1, s2, v1, v2, a, a2), base);
}

__device__ __forceinline__ float fast_exp2(float x) { return __builtin_amdgcn_exp2f(x); }

constexpr int kStat = 16;   // per-column sufficient statistics of the M-step
constexpr int kHg = 27;     // per-column normal-equation contribution (21 + 6)

// M-step sufficient statistics of one (detected spot p, model spot) pair with
// plan weight Q, at the current column geometry cC (detector frame).  With
// delta = p - s, d = v + delta, tau = |d|, rhat = d / tau, P = I - rhat rhat^T:
//   a[0] += Q, a[1..3] += Q (rhat - r), a[4..9] += Q P / tau^2, a[10..15] += Q P / tau
// where rhat - r = (delta - r dl) / tau, dl = |d| - |v| = (2 v.delta + |delta|^2) / (|d| + |v|),
// is formed without cancellation.  vlen = |v|, (rn, r1, r2) = v / |v|.
__device__ __forceinline__ void accumulate_stats(float *a, float Q, float p1, float p2,
                                                 const Col8 &cC, float vlen, float rn, float r1,
                                                 float r2) {
    const float dy = p1 - cC.s1, dz = p2 - cC.s2;
    const float h0u = cC.vn, h1u = cC.v1 + dy, h2u = cC.v2 + dz;
    const float dd = fmaf(h2u, h2u, fmaf(h1u, h1u, h0u * h0u));
    const float itau = __builtin_amdgcn_rsqf(dd);
    const float tau = dd * itau;
    const float dl = fmaf(2.0f, fmaf(cC.v2, dz, cC.v1 * dy), fmaf(dz, dz, dy * dy)) *
                     __builtin_amdgcn_rcpf(tau + vlen);
    const float e0 = (-rn * dl) * itau;
    const float e1 = fmaf(-r1, dl, dy) * itau;
    const float e2 = fmaf(-r2, dl, dz) * itau;
    const float h0 = h0u * itau, h1 = h1u * itau, h2 = h2u * itau;
    const float wa = Q * itau * itau, wb = Q * itau;
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

// The statistics of one pair alone (a[] is overwritten).
__device__ __forceinline__ void stats_of(float *a, float Q, float p1, float p2,
                                                 const Col8 &cC, float vlen, float rn, float r1,
                                                 float r2) {
    const float dy = p1 - cC.s1, dz = p2 - cC.s2;
    const float h0u = cC.vn, h1u = cC.v1 + dy, h2u = cC.v2 + dz;
    const float dd = fmaf(h2u, h2u, fmaf(h1u, h1u, h0u * h0u));
    const float itau = __builtin_amdgcn_rsqf(dd);
    const float tau = dd * itau;
    const float dl = fmaf(2.0f, fmaf(cC.v2, dz, cC.v1 * dy), fmaf(dz, dz, dy * dy)) *
                     __builtin_amdgcn_rcpf(tau + vlen);
    const float e0 = (-rn * dl) * itau;
    const float e1 = fmaf(-r1, dl, dy) * itau;
    const float e2 = fmaf(-r2, dl, dz) * itau;
    const float h0 = h0u * itau, h1 = h1u * itau, h2 = h2u * itau;
    const float wa = Q * itau * itau, wb = Q * itau;
    const float P00 = fmaf(-h0, h0, 1.0f), P01 = -h0 * h1, P02 = -h0 * h2;
    const float P11 = fmaf(-h1, h1, 1.0f), P12 = -h1 * h2, P22 = fmaf(-h2, h2, 1.0f);
    a[0] = Q;
    a[1] = Q * e0;
    a[2] = Q * e1;
    a[3] = Q * e2;
    a[4] = wa * P00;
    a[5] = wa * P01;
    a[6] = wa * P02;
    a[7] = wa * P11;
    a[8] = wa * P12;
    a[9] = wa * P22;
    a[10] = wb * P00;
    a[11] = wb * P01;
    a[12] = wb * P02;
    a[13] = wb * P11;
    a[14] = wb * P12;
    a[15] = wb * P22;
}

// FP64 contribution of one model spot (plane m, grain n, block b) to its
// grain's Gauss-Newton normal equations, from the column statistics s64
// (detector frame, see accumulate_stats).  Residual rho = D (rhat - r);
// Jacobians (from Eqs. ray_mnt and s_mnt, left perturbation
// R <- exp([omega]_x) R): d rho/d x = -(D/tau) P Gt, d rho/d omega = -D K with
// K = 2 (u e^T + (u.e) I) Gt [R w]_x, u = Gt R w.  Hence
//   H_ww = D^2 S0 K^T K, H_xx = D^2 Gt^T A Gt, H_xw = D^2 Gt^T B K,
//   g_w = -D^2 K^T e,    g_x = D^2 Gt^T B r,
// written as the 21 upper-triangle entries of H (theta = (omega, x)) and g.
// Invalid ids contribute zeros.
__device__ inline void column_normal_equations(const GeomF &Gm, const float *W, int n_planes,
                                               const GrainF *grains, int n_grains, int m, int n,
                                               int b, const double *s64, float rn, float r1,
                                               float r2, double D2, double *o) {
    if (m < 0 || m >= n_planes || n < 0 || n >= n_grains || b < 0 || b >= Gm.n_rot * Gm.n_det) {
        for (int k = 0; k < kHg; ++k) o[k] = 0.0;
        return;
    }
    const int t = b / Gm.n_det, d = b - t * Gm.n_det;
    const DetF &Dt = Gm.det[d];
    double Mf[3][3];  // columns: normal, axis1, axis2 (lab = Mf * local)
    for (int a_ = 0; a_ < 3; ++a_) {
        Mf[a_][0] = Dt.n[a_];
        Mf[a_][1] = Dt.a1[a_];
        Mf[a_][2] = Dt.a2[a_];
    }
    const double cs = Gm.cs[t][0], sn = Gm.cs[t][1];
    const double Gt[3][3] = {{cs, -sn, 0.0}, {sn, cs, 0.0}, {0.0, 0.0, 1.0}};
    const float *R = grains[n].R;
    double vs[3];
    for (int a_ = 0; a_ < 3; ++a_)
        vs[a_] = static_cast<double>(R[3 * a_]) * W[3 * m] +
                 static_cast<double>(R[3 * a_ + 1]) * W[3 * m + 1] +
                 static_cast<double>(R[3 * a_ + 2]) * W[3 * m + 2];
    double u[3];
    for (int a_ = 0; a_ < 3; ++a_) u[a_] = Gt[a_][0] * vs[0] + Gt[a_][1] * vs[1] + Gt[a_][2] * vs[2];
    const double Vx[3][3] = {{0.0, -vs[2], vs[1]}, {vs[2], 0.0, -vs[0]}, {-vs[1], vs[0], 0.0}};
    double GV[3][3], Kj[3][3];
    for (int a_ = 0; a_ < 3; ++a_)
        for (int b_ = 0; b_ < 3; ++b_)
            GV[a_][b_] = Gt[a_][0] * Vx[0][b_] + Gt[a_][1] * Vx[1][b_] + Gt[a_][2] * Vx[2][b_];
    for (int a_ = 0; a_ < 3; ++a_)
        for (int b_ = 0; b_ < 3; ++b_) Kj[a_][b_] = 2.0 * (u[a_] * GV[0][b_] + u[0] * GV[a_][b_]);
    const double S0 = s64[0];
    const double eloc[3] = {s64[1], s64[2], s64[3]};
    const double Aloc[3][3] = {{s64[4], s64[5], s64[6]}, {s64[5], s64[7], s64[8]}, {s64[6], s64[8], s64[9]}};
    const double Bloc[3][3] = {{s64[10], s64[11], s64[12]}, {s64[11], s64[13], s64[14]}, {s64[12], s64[14], s64[15]}};
    const double rloc[3] = {rn, r1, r2};
    double el[3], rl[3], Al[3][3], Bl[3][3], T1[3][3], T2[3][3];
    for (int a_ = 0; a_ < 3; ++a_) {
        el[a_] = Mf[a_][0] * eloc[0] + Mf[a_][1] * eloc[1] + Mf[a_][2] * eloc[2];
        rl[a_] = Mf[a_][0] * rloc[0] + Mf[a_][1] * rloc[1] + Mf[a_][2] * rloc[2];
    }
    for (int a_ = 0; a_ < 3; ++a_)
        for (int b_ = 0; b_ < 3; ++b_) {
            T1[a_][b_] = Mf[a_][0] * Aloc[0][b_] + Mf[a_][1] * Aloc[1][b_] + Mf[a_][2] * Aloc[2][b_];
            T2[a_][b_] = Mf[a_][0] * Bloc[0][b_] + Mf[a_][1] * Bloc[1][b_] + Mf[a_][2] * Bloc[2][b_];
        }
    for (int a_ = 0; a_ < 3; ++a_)
        for (int b_ = 0; b_ < 3; ++b_) {
            Al[a_][b_] = T1[a_][0] * Mf[b_][0] + T1[a_][1] * Mf[b_][1] + T1[a_][2] * Mf[b_][2];
            Bl[a_][b_] = T2[a_][0] * Mf[b_][0] + T2[a_][1] * Mf[b_][1] + T2[a_][2] * Mf[b_][2];
        }
    double GA[3][3], GB[3][3];
    for (int a_ = 0; a_ < 3; ++a_)
        for (int b_ = 0; b_ < 3; ++b_) {
            GA[a_][b_] = Gt[0][a_] * Al[0][b_] + Gt[1][a_] * Al[1][b_] + Gt[2][a_] * Al[2][b_];
            GB[a_][b_] = Gt[0][a_] * Bl[0][b_] + Gt[1][a_] * Bl[1][b_] + Gt[2][a_] * Bl[2][b_];
        }
    double H[6][6], gv[6];
    for (int a_ = 0; a_ < 3; ++a_)
        for (int b_ = 0; b_ < 3; ++b_) {
            double ww = 0.0, xx = 0.0, xw = 0.0;
            for (int c_ = 0; c_ < 3; ++c_) {
                ww += Kj[c_][a_] * Kj[c_][b_];
                xx += GA[a_][c_] * Gt[c_][b_];
                xw += GB[a_][c_] * Kj[c_][b_];
            }
            H[a_][b_] = D2 * S0 * ww;
            H[3 + a_][3 + b_] = D2 * xx;
            H[3 + a_][b_] = D2 * xw;
            H[b_][3 + a_] = D2 * xw;
        }
    for (int a_ = 0; a_ < 3; ++a_) {
        double gw = 0.0, gx = 0.0;
        for (int c_ = 0; c_ < 3; ++c_) {
            gw += Kj[c_][a_] * el[c_];
            gx += GB[a_][c_] * rl[c_];
        }
        gv[a_] = -D2 * gw;
        gv[3 + a_] = D2 * gx;
    }
    int q = 0;
    for (int a_ = 0; a_ < 6; ++a_)
        for (int b_ = a_; b_ < 6; ++b_) o[q++] = H[a_][b_];
    for (int a_ = 0; a_ < 6; ++a_) o[q++] = gv[a_];
}

// Gauss-Newton step of one grain from its summed normal equations acc
// (21 upper-triangle entries of H, then g): (H + mu I) step = -g with
// mu = mu_rel tr(H) / 6, solved by FP64 Cholesky; R <- exp([omega]_x) R as the
// quaternion product dq * q, x <- x + dx.  A grain without weight (tr H ~ 0)
// or with a non-positive pivot keeps its parameters (step 0).
__device__ inline void gn_solve_apply(const double *acc, double mu_rel, double *q, double *x,
                                      GrainF *gf, double *step_norm) {
    double H[6][6], gv[6];
    int c = 0;
#pragma unroll
    for (int a = 0; a < 6; ++a)
#pragma unroll
        for (int b = a; b < 6; ++b) {
            H[a][b] = acc[c];
            H[b][a] = acc[c];
            ++c;
        }
#pragma unroll
    for (int a = 0; a < 6; ++a) gv[a] = acc[21 + a];
    double tr = 0.0;
#pragma unroll
    for (int a = 0; a < 6; ++a) tr += H[a][a];
    double step[6] = {0, 0, 0, 0, 0, 0};
    bool ok = tr > 1e-300 && isfinite(tr);
    if (ok) {
        const double mu = mu_rel * tr / 6.0;
        for (int a = 0; a < 6; ++a) H[a][a] += mu;
        // fully unrolled (the factors stay in registers): a non-positive
        // pivot clears ok and the factorisation runs on with a unit pivot,
        // its result discarded
        double L[6][6] = {};
#pragma unroll
        for (int a = 0; a < 6; ++a) {
#pragma unroll
            for (int b = 0; b <= a; ++b) {
                double s = H[a][b];
#pragma unroll
                for (int k = 0; k < b; ++k) s -= L[a][k] * L[b][k];
                if (a == b) {
                    ok = ok && s > 0.0;
                    L[a][a] = sqrt(s > 0.0 ? s : 1.0);
                } else {
                    L[a][b] = s / L[b][b];
                }
            }
        }
        if (ok) {
            double y[6];
#pragma unroll
            for (int a = 0; a < 6; ++a) {
                double s = -gv[a];
#pragma unroll
                for (int k = 0; k < a; ++k) s -= L[a][k] * y[k];
                y[a] = s / L[a][a];
            }
#pragma unroll
            for (int a = 5; a >= 0; --a) {
                double s = y[a];
#pragma unroll
                for (int k = a + 1; k < 6; ++k) s -= L[k][a] * step[k];
                step[a] = s / L[a][a];
            }
        }
    }
    if (!ok) {
        for (int a = 0; a < 6; ++a) step[a] = 0.0;
    }
    // R <- exp([w]_x) R as the quaternion product dq * q
    double qw = q[0], qa = q[1], qb = q[2], qc = q[3];
    const double th = sqrt(step[0] * step[0] + step[1] * step[1] + step[2] * step[2]);
    if (th > 0.0) {
        const double h = 0.5 * th, sh = sin(h) / th;
        const double dw = cos(h), da = step[0] * sh, db = step[1] * sh, dc = step[2] * sh;
        const double nw = dw * qw - da * qa - db * qb - dc * qc;
        const double na = dw * qa + da * qw + db * qc - dc * qb;
        const double nb = dw * qb - da * qc + db * qw + dc * qa;
        const double nc = dw * qc + da * qb - db * qa + dc * qw;
        qw = nw; qa = na; qb = nb; qc = nc;
    }
    double nrm = sqrt(qw * qw + qa * qa + qb * qb + qc * qc);
    qw /= nrm; qa /= nrm; qb /= nrm; qc /= nrm;
    if (qw < 0) { qw = -qw; qa = -qa; qb = -qb; qc = -qc; }
    q[0] = qw; q[1] = qa; q[2] = qb; q[3] = qc;
    for (int a = 0; a < 3; ++a) x[a] += step[3 + a];
    const double Rm[9] = {1 - 2 * (qb * qb + qc * qc), 2 * (qa * qb - qw * qc), 2 * (qa * qc + qw * qb),
                          2 * (qa * qb + qw * qc), 1 - 2 * (qa * qa + qc * qc), 2 * (qb * qc - qw * qa),
                          2 * (qa * qc - qw * qb), 2 * (qb * qc + qw * qa), 1 - 2 * (qa * qa + qb * qb)};
    for (int k = 0; k < 9; ++k) gf->R[k] = static_cast<float>(Rm[k]);
    for (int k = 0; k < 3; ++k) gf->x[k] = static_cast<float>(x[k]);
    if (step_norm) {
        double s = 0.0;
        for (int a = 0; a < 6; ++a) s += step[a] * step[a];
        *step_norm = sqrt(s);
    }
}

// ---------------------------------------------------------------- coordinate-descent M-step

// The paper's own M-step (App. B): LauePosNewton on x with R fixed, then
// LaueRotMM on R at the new x, both maximising F = sum Q rhat^T r.
constexpr int kPosStat = 9;        // per-column statistics of LauePosNewton
constexpr int kDirStat = 3;        // per-column statistics of LaueRotMM
constexpr int kMaxPlanesMM = 1024; // planes a grain's MM can hold (LDS)

// LauePosNewton statistics of one pair (detector frame).  With h = rhat,
// eps = rhat - r (formed without cancellation as in accumulate_stats) and
// eta = |eps|^2 / 2 = 1 - rhat.r, Eqs. xgrad and xhess per pair become
//   dF/dy   = (eps - eta h) / tau
//   d2F/dy2 = -[(1 - eta) I + (3 eta - 1) h h^T - (eps h^T + h eps^T)] / tau^2
// (no term cancels: the small rhat.r - 1 and P r enter through eps and eta).
//   a[0..2] += Q (eps - eta h) / tau,
//   a[3..8] += Q [(1 - eta) I + (3 eta - 1) h h^T - (eps h^T + h eps^T)] / tau^2
// (upper triangle 00, 01, 02, 11, 12, 22).
__device__ __forceinline__ void accumulate_pos(float *a, float Q, float p1, float p2, const Col8 &cC, float vlen,
                                               float rn, float r1, float r2) {
    const float dy = p1 - cC.s1, dz = p2 - cC.s2;
    const float h0u = cC.vn, h1u = cC.v1 + dy, h2u = cC.v2 + dz;
    const float dd = fmaf(h2u, h2u, fmaf(h1u, h1u, h0u * h0u));
    const float itau = __builtin_amdgcn_rsqf(dd);
    const float tau = dd * itau;
    const float dl = fmaf(2.0f, fmaf(cC.v2, dz, cC.v1 * dy), fmaf(dz, dz, dy * dy)) *
                     __builtin_amdgcn_rcpf(tau + vlen);
    const float e0 = (-rn * dl) * itau;
    const float e1 = fmaf(-r1, dl, dy) * itau;
    const float e2 = fmaf(-r2, dl, dz) * itau;
    const float h0 = h0u * itau, h1 = h1u * itau, h2 = h2u * itau;
    const float eta = 0.5f * fmaf(e2, e2, fmaf(e1, e1, e0 * e0));
    const float wb = Q * itau, wa = wb * itau;
    a[0] = fmaf(wb, fmaf(-eta, h0, e0), a[0]);
    a[1] = fmaf(wb, fmaf(-eta, h1, e1), a[1]);
    a[2] = fmaf(wb, fmaf(-eta, h2, e2), a[2]);
    const float c1 = 1.0f - eta, c3 = fmaf(3.0f, eta, -1.0f);
    a[3] = fmaf(wa, fmaf(c3 * h0, h0, fmaf(-2.0f * e0, h0, c1)), a[3]);
    a[4] = fmaf(wa, fmaf(c3 * h0, h1, -fmaf(e0, h1, h0 * e1)), a[4]);
    a[5] = fmaf(wa, fmaf(c3 * h0, h2, -fmaf(e0, h2, h0 * e2)), a[5]);
    a[6] = fmaf(wa, fmaf(c3 * h1, h1, fmaf(-2.0f * e1, h1, c1)), a[6]);
    a[7] = fmaf(wa, fmaf(c3 * h1, h2, -fmaf(e1, h2, h1 * e2)), a[7]);
    a[8] = fmaf(wa, fmaf(c3 * h2, h2, fmaf(-2.0f * e2, h2, c1)), a[8]);
}

// LaueRotMM statistics of one pair (detector frame): a[0..2] += Q rhat.
__device__ __forceinline__ void accumulate_dir(float *a, float Q, float p1, float p2, const Col8 &cC) {
    const float dy = p1 - cC.s1, dz = p2 - cC.s2;
    const float h0u = cC.vn, h1u = cC.v1 + dy, h2u = cC.v2 + dz;
    const float dd = fmaf(h2u, h2u, fmaf(h1u, h1u, h0u * h0u));
    const float wq = Q * __builtin_amdgcn_rsqf(dd);
    a[0] = fmaf(wq, h0u, a[0]);
    a[1] = fmaf(wq, h1u, a[1]);
    a[2] = fmaf(wq, h2u, a[2]);
}

// Detector frame (lab = Mf local, columns normal, axis1, axis2) and the
// rotation-stage matrix Gt (y = Gt x) of block b; false for an invalid block.
__device__ inline bool column_frames(const GeomF &Gm, int b, double Mf[3][3], double Gt[3][3]) {
    if (b < 0 || b >= Gm.n_rot * Gm.n_det) return false;
    const int t = b / Gm.n_det, d = b - t * Gm.n_det;
    const DetF &Dt = Gm.det[d];
    for (int a_ = 0; a_ < 3; ++a_) {
        Mf[a_][0] = Dt.n[a_];
        Mf[a_][1] = Dt.a1[a_];
        Mf[a_][2] = Dt.a2[a_];
    }
    const double cs = Gm.cs[t][0], sn = Gm.cs[t][1];
    Gt[0][0] = cs;  Gt[0][1] = -sn; Gt[0][2] = 0.0;
    Gt[1][0] = sn;  Gt[1][1] = cs;  Gt[1][2] = 0.0;
    Gt[2][0] = 0.0; Gt[2][1] = 0.0; Gt[2][2] = 1.0;
    return true;
}

// One column's FP64 contribution to its grain's LauePosNewton system, in the
// sample frame: H_x = Gt^T (Mf Hy Mf^T) Gt and g_x = Gt^T Mf gy from the
// statistics of accumulate_pos.  o[0..5]: H_x (00, 01, 02, 11, 12, 22),
// o[6..8]: g_x.  Invalid ids contribute zeros.
__device__ inline void column_pos_newton(const GeomF &Gm, int n_grains, int n, int b, const double *s64, double *o) {
    double Mf[3][3], Gt[3][3];
    if (n < 0 || n >= n_grains || !column_frames(Gm, b, Mf, Gt)) {
        for (int k = 0; k < kPosStat; ++k) o[k] = 0.0;
        return;
    }
    const double S[3][3] = {{s64[3], s64[4], s64[5]}, {s64[4], s64[6], s64[7]}, {s64[5], s64[7], s64[8]}};
    double T[3][3], L[3][3], gl[3];
    for (int a_ = 0; a_ < 3; ++a_) {
        gl[a_] = Mf[a_][0] * s64[0] + Mf[a_][1] * s64[1] + Mf[a_][2] * s64[2];
        for (int b_ = 0; b_ < 3; ++b_) T[a_][b_] = Mf[a_][0] * S[0][b_] + Mf[a_][1] * S[1][b_] + Mf[a_][2] * S[2][b_];
    }
    for (int a_ = 0; a_ < 3; ++a_)
        for (int b_ = 0; b_ < 3; ++b_) L[a_][b_] = T[a_][0] * Mf[b_][0] + T[a_][1] * Mf[b_][1] + T[a_][2] * Mf[b_][2];
    double GL[3][3], H[3][3];
    for (int a_ = 0; a_ < 3; ++a_)
        for (int b_ = 0; b_ < 3; ++b_) GL[a_][b_] = Gt[0][a_] * L[0][b_] + Gt[1][a_] * L[1][b_] + Gt[2][a_] * L[2][b_];
    for (int a_ = 0; a_ < 3; ++a_)
        for (int b_ = 0; b_ < 3; ++b_) H[a_][b_] = -(GL[a_][0] * Gt[0][b_] + GL[a_][1] * Gt[1][b_] + GL[a_][2] * Gt[2][b_]);
    o[0] = H[0][0]; o[1] = H[0][1]; o[2] = H[0][2]; o[3] = H[1][1]; o[4] = H[1][2]; o[5] = H[2][2];
    for (int a_ = 0; a_ < 3; ++a_) o[6 + a_] = Gt[0][a_] * gl[0] + Gt[1][a_] * gl[1] + Gt[2][a_] * gl[2];
}

// One column's FP64 contribution to M0 of its (grain, plane) (Eq. M0):
// -Gt^T (q e^T + e q^T) Gt with q = sum_i Q rhat in the lab and e the beam
// direction (1, 0, 0).  o[0..5]: 00, 01, 02, 11, 12, 22.
__device__ inline void column_rot_m0(const GeomF &Gm, int b, const double *s64, double *o) {
    double Mf[3][3], Gt[3][3];
    if (!column_frames(Gm, b, Mf, Gt)) {
        for (int k = 0; k < 6; ++k) o[k] = 0.0;
        return;
    }
    double ql[3], c[3], f[3];
    for (int a_ = 0; a_ < 3; ++a_) ql[a_] = Mf[a_][0] * s64[0] + Mf[a_][1] * s64[1] + Mf[a_][2] * s64[2];
    for (int a_ = 0; a_ < 3; ++a_) {
        c[a_] = Gt[0][a_] * ql[0] + Gt[1][a_] * ql[1] + Gt[2][a_] * ql[2];
        f[a_] = Gt[0][a_];
    }
    o[0] = -2.0 * c[0] * f[0];
    o[1] = -(c[0] * f[1] + f[0] * c[1]);
    o[2] = -(c[0] * f[2] + f[0] * c[2]);
    o[3] = -2.0 * c[1] * f[1];
    o[4] = -(c[1] * f[2] + f[1] * c[2]);
    o[5] = -2.0 * c[2] * f[2];
}

// Smallest eigenvalue of a symmetric 3x3 matrix (00, 01, 02, 11, 12, 22),
// by the trigonometric solution of its characteristic cubic.  FP64.
__device__ inline double sym3_min_eig(const double *m) {
    const double p1 = m[1] * m[1] + m[2] * m[2] + m[4] * m[4];
    const double tr3 = (m[0] + m[3] + m[5]) / 3.0;
    if (p1 == 0.0) return fmin(m[0], fmin(m[3], m[5]));
    const double d0 = m[0] - tr3, d1 = m[3] - tr3, d2 = m[5] - tr3;
    const double p = sqrt((d0 * d0 + d1 * d1 + d2 * d2 + 2.0 * p1) / 6.0);
    const double ip = 1.0 / p;
    const double b00 = d0 * ip, b11 = d1 * ip, b22 = d2 * ip, b01 = m[1] * ip, b02 = m[2] * ip, b12 = m[4] * ip;
    const double det = b00 * (b11 * b22 - b12 * b12) - b01 * (b01 * b22 - b12 * b02) + b02 * (b01 * b12 - b11 * b02);
    const double r = fmin(1.0, fmax(-1.0, 0.5 * det));
    const double phi = acos(r) / 3.0;
    return tr3 + 2.0 * p * cos(phi + 2.0943951023931957);
}

// Largest-eigenvalue eigenvector of a symmetric 4x4 matrix (cyclic Jacobi, FP64).
__device__ inline void sym4_top_eigvec(double A[4][4], double v[4]) {
    double V[4][4] = {{1, 0, 0, 0}, {0, 1, 0, 0}, {0, 0, 1, 0}, {0, 0, 0, 1}};
    for (int sweep = 0; sweep < 12; ++sweep) {
        double off = 0.0, dia = 0.0;
        for (int p = 0; p < 4; ++p) {
            dia += A[p][p] * A[p][p];
            for (int q = p + 1; q < 4; ++q) off += A[p][q] * A[p][q];
        }
        if (off <= 1e-30 * dia) break;
        for (int p = 0; p < 3; ++p)
            for (int q = p + 1; q < 4; ++q) {
                if (fabs(A[p][q]) < 1e-300) continue;
                const double th = (A[q][q] - A[p][p]) / (2.0 * A[p][q]);
                const double t = (th >= 0 ? 1.0 : -1.0) / (fabs(th) + sqrt(th * th + 1.0));
                const double c = 1.0 / sqrt(t * t + 1.0), s = t * c;
                for (int k = 0; k < 4; ++k) {
                    const double kp = A[k][p], kq = A[k][q];
                    A[k][p] = c * kp - s * kq;
                    A[k][q] = s * kp + c * kq;
                }
                for (int k = 0; k < 4; ++k) {
                    const double pk = A[p][k], qk = A[q][k];
                    A[p][k] = c * pk - s * qk;
                    A[q][k] = s * pk + c * qk;
                }
                for (int k = 0; k < 4; ++k) {
                    const double kp = V[k][p], kq = V[k][q];
                    V[k][p] = c * kp - s * kq;
                    V[k][q] = s * kp + c * kq;
                }
            }
    }
    int best = 0;
    for (int i = 1; i < 4; ++i)
        if (A[i][i] > A[best][best]) best = i;
    for (int k = 0; k < 4; ++k) v[k] = V[k][best];
}

// Wahba's problem (App. A) from B = sum_k w_k a_k b_k^T: the rotation R
// minimising sum_k w_k ||a_k - R b_k||^2, through Davenport's q-method (the
// same minimiser as the SVD form of Alg. Wahba): the optimal unit quaternion
// (w >= 0) is the top eigenvector of K = [[tr B, z^T], [z, B + B^T - tr(B) I]],
// z = (B21 - B12, B02 - B20, B10 - B01).
__device__ inline void wahba_quat_B(const double B[3][3], double *q) {
    const double tr = B[0][0] + B[1][1] + B[2][2];
    const double z[3] = {B[2][1] - B[1][2], B[0][2] - B[2][0], B[1][0] - B[0][1]};
    double K[4][4];
    K[0][0] = tr;
    for (int i = 0; i < 3; ++i) {
        K[0][1 + i] = z[i];
        K[1 + i][0] = z[i];
        for (int j = 0; j < 3; ++j) K[1 + i][1 + j] = B[i][j] + B[j][i] - (i == j ? tr : 0.0);
    }
    sym4_top_eigvec(K, q);
    const double nrm = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
    const double sg = q[0] < 0 ? -1.0 : 1.0;
    for (int k = 0; k < 4; ++k) q[k] = sg * q[k] / nrm;
}

// Row-major rotation matrix of a unit quaternion (w, x, y, z).
__device__ inline void quat_R(const double *q, double *R) {
    const double w = q[0], a = q[1], b = q[2], c = q[3];
    R[0] = 1 - 2 * (b * b + c * c); R[1] = 2 * (a * b - w * c);     R[2] = 2 * (a * c + w * b);
    R[3] = 2 * (a * b + w * c);     R[4] = 1 - 2 * (a * a + c * c); R[5] = 2 * (b * c - w * a);
    R[6] = 2 * (a * c - w * b);     R[7] = 2 * (b * c + w * a);     R[8] = 1 - 2 * (a * a + b * b);
}

// Workspace of the enumerate count/scan (forward.hip).
struct EnumWs {
    GeomF *geom;
    GrainF *grains;
    int *counts;
    int64_t *offs;      // exclusive scan of counts in (t, d, n) order, L + 1 entries
    int64_t *blk;       // per-block offsets (n_blocks + 1)
    unsigned *kmask;    // kept-plane bits per (t, n) item and detector (w32 words each), or NULL
    int w32;
    bool mask_ready;    // set by enumerate_count when it wrote kmask for these grains
};
// n_planes sizes the kept-plane bits (the kernel's limit of 1024 when unknown)
size_t carve_enum(Carver &cv, EnumWs &w, const laue_geometry *g, int n_grains, int n_planes = 1024);
int enumerate_count(const laue_geometry *geom, const laue_planes *planes, const laue_grains *grains,
                    int merge, EnumWs &w, std::vector<int64_t> &host_blk, int64_t *total,
                    hipStream_t s);
int prep_grains(const laue_grains *g, GrainF *dst, hipStream_t s);
int launch_eval(const GeomF *dG, const laue_planes *pl, const GrainF *dgr, int n_grains,
                const int *plane, const int *grain, const int *block, int64_t n, float *s1,
                float *s2, float *vn, float *v1, float *v2, float *lam, Col8 *cols, hipStream_t s);
// Write pass of the enumerate (ids only) after enumerate_count on the same
// workspace; n_total is the count's total (the length of the id arrays).
int launch_enumerate_ids(const laue_geometry *geom, const laue_planes *planes, EnumWs &w, int N,
                         int merge, int64_t n_total, int *plane, int *grain, int *block, hipStream_t s);
int validate_planes(const laue_planes *p);
int validate_grains(const laue_grains *g);
// exclusive scan of L ints into L + 1 int64 (one workgroup)
int launch_scan(const int *in, int64_t *out, int64_t L, hipStream_t s);

// Philox4x32-10 (Salmon et al., SC'11), from its published definition.
__device__ __forceinline__ void philox(uint32_t c[4], uint32_t k0, uint32_t k1) {
    for (int r = 0; r < 10; ++r) {
        uint64_t p0 = static_cast<uint64_t>(0xD2511F53u) * c[0];
        uint64_t p1 = static_cast<uint64_t>(0xCD9E8D57u) * c[2];
        uint32_t hi0 = static_cast<uint32_t>(p0 >> 32), lo0 = static_cast<uint32_t>(p0);
        uint32_t hi1 = static_cast<uint32_t>(p1 >> 32), lo1 = static_cast<uint32_t>(p1);
        uint32_t n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
        c[0] = n0;
        c[1] = lo1;
        c[2] = n2;
        c[3] = lo0;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
}


// Wave-wide (64-lane) reductions in a fixed butterfly order (deterministic).
__device__ __forceinline__ double wave_sum(double v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}
__device__ __forceinline__ double wave_max(double v) {
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    return v;
}

}  // namespace laue
