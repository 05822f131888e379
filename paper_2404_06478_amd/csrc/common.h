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
__device__ __forceinline__ float entry_exponent(float p1, float p2, float s1, float s2, float v1,
                                                float v2, float a, float a2, float K, float base) {
    const float dy = p1 - s1;
    const float dz = p2 - s2;
    const float e = fmaf(dz, dz, dy * dy);        // |delta|^2
    const float b = fmaf(v2, dz, v1 * dy);        // v.delta
    const float x2 = fmaf(a, e, -(b * b));        // |v x delta|^2
    const float vdd = a + b;                      // v.d
    const float w = fmaf(2.0f, b, e);             // |d|^2 - |v|^2
    const float P = fmaf(a, w, a2);               // |v|^2 |d|^2
    const float den = fmaf(vdd, __builtin_amdgcn_sqrtf(P), P);
    const float cp = x2 * __builtin_amdgcn_rcpf(den);
    return fmaf(-K, cp, base);
}

__device__ __forceinline__ float fast_exp2(float x) { return __builtin_amdgcn_exp2f(x); }

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
