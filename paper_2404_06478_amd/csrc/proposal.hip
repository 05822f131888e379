// Learned proposal around the network: cheap-support features of spot-pair
// candidates, training labels, and selection of the best-scored fraction.
//
// Cheap support (two features per candidate): the candidate grain, placed at
// the sample centre, predicts its harmonic-free reflections (Sec. 3.3
// forward model) at two probe rotations t + floor(kT/3) mod T, k = 1, 2, away
// from the rotation its pair was drawn at; a prediction is hit when a
// detected spot of the same (rotation, detector) block lies within a radius.
// Detected spots are bucketed once into a uniform grid per block (cell side
// >= radius, so a query visits 3x3 cells).  Geometry in FP64.
//
// Selection: k = ceil(frac n) largest scores, equal scores in increasing index
// order, by a four-pass 8-bit radix select on order-preserving integer keys,
// then two exclusive scans (rank among equal keys, output position).
#include <algorithm>
#include <cmath>
#include <vector>

#include "common.h"

namespace laue {

namespace {

constexpr int kMaxGridSide = 256;

struct SupportGrid {
    int nc;          // cells per side
    double half;     // grid covers [-half, half]^2 in detector coordinates
    double h;        // cell side
};

__device__ __forceinline__ int grid_cell(const SupportGrid &g, double v) {
    if (!(fabs(v) <= g.half)) return v > 0.0 ? g.nc - 1 : 0;     // outside or NaN: clamp
    int c = static_cast<int>(floor((v + g.half) / g.h));
    return c < 0 ? 0 : (c >= g.nc ? g.nc - 1 : c);
}

__global__ void k_grid_count(const float *__restrict__ p1, const float *__restrict__ p2,
                             const int64_t *__restrict__ ooff, int nb, int64_t n, SupportGrid g,
                             int *__restrict__ cnt, int *__restrict__ cell_of) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int lo = 0, hi = nb;                     // block b with ooff[b] <= i < ooff[b+1]
    while (hi - lo > 1) {
        const int mid = (lo + hi) / 2;
        if (ooff[mid] <= i) lo = mid; else hi = mid;
    }
    const int c = (lo * g.nc + grid_cell(g, p2[i])) * g.nc + grid_cell(g, p1[i]);
    cell_of[i] = c;
    atomicAdd(&cnt[c], 1);
}

__global__ void k_grid_fill(const float *__restrict__ p1, const float *__restrict__ p2, int64_t n,
                            const int *__restrict__ cell_of, const int64_t *__restrict__ coff,
                            int *__restrict__ cursor, float2 *__restrict__ pts) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int c = cell_of[i];
    const int64_t pos = coff[c] + atomicAdd(&cursor[c], 1);
    pts[pos] = make_float2(p1[i], p2[i]);
}

__device__ inline void quat_R(const double *q, double R[3][3]) {
    const double n = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
    const double w = q[0] / n, x = q[1] / n, y = q[2] / n, z = q[3] / n;
    R[0][0] = 1 - 2 * (y * y + z * z); R[0][1] = 2 * (x * y - w * z);     R[0][2] = 2 * (x * z + w * y);
    R[1][0] = 2 * (x * y + w * z);     R[1][1] = 1 - 2 * (x * x + z * z); R[1][2] = 2 * (y * z - w * x);
    R[2][0] = 2 * (x * z - w * y);     R[2][1] = 2 * (y * z + w * x);     R[2][2] = 1 - 2 * (x * x + y * y);
}

// One thread per candidate.
__global__ void k_support(const laue_geometry G, const float *__restrict__ W, const float *__restrict__ Dsp,
                          const int *__restrict__ probe, int n_probe, const double *__restrict__ q,
                          const int *__restrict__ spot_a, int64_t n_cand, const int64_t *__restrict__ ooff,
                          int64_t n_obs, SupportGrid g, const int64_t *__restrict__ coff,
                          const float2 *__restrict__ pts, double radius, float *__restrict__ feat) {
    const int64_t c = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (c >= n_cand) return;
    const int nb = G.n_rot * G.n_det;
    const int a = spot_a[c];
    float *f = feat + 16 * c;
    if (a < 0 || a >= n_obs) {
        f[14] = 0.0f;
        f[15] = 0.0f;
        return;
    }
    int lo = 0, hi = nb;
    while (hi - lo > 1) {
        const int mid = (lo + hi) / 2;
        if (ooff[mid] <= a) lo = mid; else hi = mid;
    }
    const int t0 = lo / G.n_det;
    double R[3][3];
    quat_R(q + 4 * c, R);
    const double r2 = radius * radius;
    for (int k = 1; k <= 2; ++k) {
        const int t = (t0 + (k * G.n_rot) / 3) % G.n_rot;
        const double om = G.omega0 + G.domega * t, co = cos(om), so = sin(om);
        int pred = 0, hits = 0;
        for (int pi = 0; pi < n_probe; ++pi) {
            const int m = probe[pi];
            const double w0 = W[3 * m], w1 = W[3 * m + 1], w2 = W[3 * m + 2];
            const double v0 = R[0][0] * w0 + R[0][1] * w1 + R[0][2] * w2;
            const double v1 = R[1][0] * w0 + R[1][1] * w1 + R[1][2] * w2;
            const double v2 = R[2][0] * w0 + R[2][1] * w1 + R[2][2] * w2;
            const double u[3] = {co * v0 - so * v1, so * v0 + co * v1, v2};
            const double lam = 2.0 * static_cast<double>(Dsp[m]) * u[0];
            if (!(lam >= G.lambda_min && lam <= G.lambda_max)) continue;
            const double r[3] = {1.0 - 2.0 * u[0] * u[0], -2.0 * u[0] * u[1], -2.0 * u[0] * u[2]};
            for (int d = 0; d < G.n_det; ++d) {
                const laue_detector &D = G.det[d];
                const double den = r[0] * D.normal[0] + r[1] * D.normal[1] + r[2] * D.normal[2];
                if (den == 0.0) continue;
                const double tau =
                    (D.center[0] * D.normal[0] + D.center[1] * D.normal[1] + D.center[2] * D.normal[2]) / den;
                if (!(tau > 0.0)) continue;
                const double rel[3] = {tau * r[0] - D.center[0], tau * r[1] - D.center[1], tau * r[2] - D.center[2]};
                const double s1 = rel[0] * D.axis1[0] + rel[1] * D.axis1[1] + rel[2] * D.axis1[2];
                const double s2 = rel[0] * D.axis2[0] + rel[1] * D.axis2[1] + rel[2] * D.axis2[2];
                if (!(fmax(fabs(s1), fabs(s2)) < D.half_size)) continue;
                ++pred;
                const int b = t * G.n_det + d;
                const int cx = grid_cell(g, s1), cy = grid_cell(g, s2);
                bool hit = false;
                for (int yy = max(cy - 1, 0); yy <= min(cy + 1, g.nc - 1) && !hit; ++yy) {
                    const int row = (b * g.nc + yy) * g.nc;
                    const int64_t e0 = coff[row + max(cx - 1, 0)], e1 = coff[row + min(cx + 1, g.nc - 1) + 1];
                    for (int64_t e = e0; e < e1; ++e) {
                        const double dx = static_cast<double>(pts[e].x) - s1, dy = static_cast<double>(pts[e].y) - s2;
                        if (dx * dx + dy * dy <= r2) {
                            hit = true;
                            break;
                        }
                    }
                }
                hits += hit;
            }
        }
        f[13 + k] = static_cast<float>(static_cast<double>(hits) / static_cast<double>(max(pred, 1)));
    }
}

// Largest |<p, s>| over the 24 proper cubic rotations s (as quaternions: the
// 4 axis units, the 12 (+-e_a +- e_b)/sqrt 2, the 8 (+-1,+-1,+-1,+-1)/2).
__device__ inline double cubic_cos_half(const double *p) {
    double a[4] = {fabs(p[0]), fabs(p[1]), fabs(p[2]), fabs(p[3])};
    for (int i = 0; i < 3; ++i)                      // sort descending
        for (int j = 0; j < 3 - i; ++j)
            if (a[j] < a[j + 1]) { const double t = a[j]; a[j] = a[j + 1]; a[j + 1] = t; }
    const double m1 = a[0], m2 = (a[0] + a[1]) * 0.70710678118654752440, m3 = 0.5 * (a[0] + a[1] + a[2] + a[3]);
    return fmax(m1, fmax(m2, m3));
}

__global__ void k_labels(const double *__restrict__ q, const int *__restrict__ spot_a,
                         const int *__restrict__ spot_b, int64_t n_cand, const int *__restrict__ spot_grain,
                         int64_t n_obs, const double *__restrict__ qt, int n_true, double cos_half_max,
                         float *__restrict__ label, float *__restrict__ mis_deg) {
    const int64_t c = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (c >= n_cand) return;
    const int a = spot_a[c], b = spot_b[c];
    int ga = -1, gb = -2;
    if (a >= 0 && a < n_obs && b >= 0 && b < n_obs) {
        ga = spot_grain[a];
        gb = spot_grain[b];
    }
    float lab = 0.0f, mis = __builtin_inff();
    if (ga == gb && ga >= 0 && ga < n_true) {
        const double *p = qt + 4 * ga, *r = q + 4 * c;
        const double np_ = sqrt(p[0] * p[0] + p[1] * p[1] + p[2] * p[2] + p[3] * p[3]);
        const double nr = sqrt(r[0] * r[0] + r[1] * r[1] + r[2] * r[2] + r[3] * r[3]);
        // dq = conj(p) (x) r
        double dq[4];
        dq[0] = p[0] * r[0] + p[1] * r[1] + p[2] * r[2] + p[3] * r[3];
        dq[1] = p[0] * r[1] - p[1] * r[0] - p[2] * r[3] + p[3] * r[2];
        dq[2] = p[0] * r[2] + p[1] * r[3] - p[2] * r[0] - p[3] * r[1];
        dq[3] = p[0] * r[3] - p[1] * r[2] + p[2] * r[1] - p[3] * r[0];
        for (int i = 0; i < 4; ++i) dq[i] /= np_ * nr;
        const double ch = fmin(1.0, cubic_cos_half(dq));
        lab = ch >= cos_half_max ? 1.0f : 0.0f;
        mis = static_cast<float>(2.0 * acos(ch) * (180.0 / M_PI));
    }
    label[c] = lab;
    if (mis_deg) mis_deg[c] = mis;
}

// Nearest true grain of each candidate orientation: the largest cos(angle / 2)
// over the true grains and the 24 proper cubic rotations (FP64), lowest grain
// index on ties; label 1 when the angle is within max_deg.
__global__ void k_labels_nearest(const double *__restrict__ q, int64_t n_cand, const double *__restrict__ qt,
                                 int n_true, double cos_half_max, float *__restrict__ label,
                                 float *__restrict__ mis_deg, int *__restrict__ nearest) {
    const int64_t c = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (c >= n_cand) return;
    const double *r = q + 4 * c;
    const double nr = sqrt(r[0] * r[0] + r[1] * r[1] + r[2] * r[2] + r[3] * r[3]);
    double best = -2.0;
    int arg = -1;
    for (int g = 0; g < n_true; ++g) {
        const double *p = qt + 4 * g;
        const double np_ = sqrt(p[0] * p[0] + p[1] * p[1] + p[2] * p[2] + p[3] * p[3]);
        double dq[4];
        dq[0] = p[0] * r[0] + p[1] * r[1] + p[2] * r[2] + p[3] * r[3];
        dq[1] = p[0] * r[1] - p[1] * r[0] - p[2] * r[3] + p[3] * r[2];
        dq[2] = p[0] * r[2] + p[1] * r[3] - p[2] * r[0] - p[3] * r[1];
        dq[3] = p[0] * r[3] - p[1] * r[2] + p[2] * r[1] - p[3] * r[0];
        for (int i = 0; i < 4; ++i) dq[i] /= np_ * nr;
        const double ch = fmin(1.0, cubic_cos_half(dq));
        if (ch > best) {
            best = ch;
            arg = g;
        }
    }
    label[c] = arg >= 0 && best >= cos_half_max ? 1.0f : 0.0f;
    if (mis_deg) mis_deg[c] = arg >= 0 ? static_cast<float>(2.0 * acos(best) * (180.0 / M_PI)) : __builtin_inff();
    if (nearest) nearest[c] = arg;
}

// Same-grain pair k: Philox counter (k, 0, 0, 7); a = x0 mod n; b = the
// (x1 mod count)-th other spot of a's grain and rotation, in index order.
__global__ void k_same_pairs(const int64_t *__restrict__ ooff, int n_rot, int n_det,
                             const int *__restrict__ grain, int64_t n_obs, int64_t n_pairs, uint32_t k0,
                             uint32_t k1, int *__restrict__ oa, int *__restrict__ ob) {
    const int64_t k = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (k >= n_pairs) return;
    int ra = -1, rb = -1;
    if (n_obs > 0) {
        uint32_t c[4] = {static_cast<uint32_t>(k), 0u, 0u, 7u};
        philox(c, k0, k1);
        const int64_t a = c[0] % static_cast<uint32_t>(n_obs);
        const int g = grain[a];
        if (g >= 0) {
            int lo = 0, hi = n_rot * n_det;
            while (hi - lo > 1) {
                const int mid = (lo + hi) / 2;
                if (ooff[mid] <= a) lo = mid; else hi = mid;
            }
            const int t = lo / n_det;
            const int64_t s0 = ooff[t * n_det], s1 = ooff[(t + 1) * n_det];
            uint32_t cnt = 0;
            for (int64_t i = s0; i < s1; ++i) cnt += (i != a && grain[i] == g);
            if (cnt > 0) {
                uint32_t r = c[1] % cnt;
                for (int64_t i = s0; i < s1; ++i)
                    if (i != a && grain[i] == g) {
                        if (r == 0) {
                            ra = static_cast<int>(a);
                            rb = static_cast<int>(i);
                            break;
                        }
                        --r;
                    }
            }
        }
    }
    oa[k] = ra;
    ob[k] = rb;
}

// ---------------------------------------------------------------- top-k select

__device__ __forceinline__ uint32_t score_key(float f) {
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7fffffffu) > 0x7f800000u) return 0u;                  // NaN ranks last
    if (u == 0x80000000u) u = 0u;                                    // -0 equals +0
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}

struct SelState {
    uint32_t prefix, mask;
    int64_t krem;
};

__global__ void k_sel_init(SelState *st, int64_t k, uint32_t *hist) {
    st->prefix = 0u;
    st->mask = 0u;
    st->krem = k;
    for (int i = 0; i < 256; ++i) hist[i] = 0u;
}

__global__ __launch_bounds__(256) void k_sel_hist(const float *__restrict__ score, int64_t n,
                                                  const SelState *__restrict__ st, int shift,
                                                  uint32_t *__restrict__ hist) {
    __shared__ uint32_t h[256];
    h[threadIdx.x] = 0u;
    __syncthreads();
    const uint32_t prefix = st->prefix, mask = st->mask;
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x; i < n;
         i += static_cast<int64_t>(gridDim.x) * 256) {
        const uint32_t key = score_key(score[i]);
        if ((key & mask) == prefix) atomicAdd(&h[(key >> shift) & 0xffu], 1u);
    }
    __syncthreads();
    if (h[threadIdx.x]) atomicAdd(&hist[threadIdx.x], h[threadIdx.x]);
}

__global__ void k_sel_pick(SelState *st, int shift, uint32_t *hist) {
    int64_t cum = 0;
    int pick = 0;
    for (int b = 255; b >= 0; --b) {
        if (cum + hist[b] >= st->krem) {
            pick = b;
            break;
        }
        cum += hist[b];
    }
    st->krem -= cum;
    st->prefix |= static_cast<uint32_t>(pick) << shift;
    st->mask |= 0xffu << shift;
    for (int i = 0; i < 256; ++i) hist[i] = 0u;
}

__global__ void k_sel_eq(const float *__restrict__ score, int64_t n, const SelState *__restrict__ st,
                         int *__restrict__ flag) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n) flag[i] = score_key(score[i]) == st->prefix;
}

__global__ void k_sel_take(const float *__restrict__ score, int64_t n, const SelState *__restrict__ st,
                           const int64_t *__restrict__ eq_rank, int *__restrict__ flag) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint32_t key = score_key(score[i]);
    flag[i] = key > st->prefix || (key == st->prefix && eq_rank[i] < st->krem);
}

__global__ void k_sel_write(const int *__restrict__ flag, const int64_t *__restrict__ pos, int64_t n,
                            int64_t k, int32_t *__restrict__ out) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n && flag[i] && pos[i] < k) out[pos[i]] = static_cast<int32_t>(i);
}

struct SupportWs {
    int64_t *ooff;
    int *probe;
    int *cnt;
    int *cell_of;
    int64_t *coff;
    float2 *pts;
};

SupportGrid make_grid(const laue_geometry *g, double radius) {
    double half = 0.0;
    for (int d = 0; d < g->n_det; ++d) half = std::max(half, g->det[d].half_size);
    SupportGrid sg;
    sg.half = half;
    sg.nc = static_cast<int>(std::min<double>(kMaxGridSide, std::max(1.0, std::floor(2.0 * half / radius))));
    sg.h = 2.0 * half / sg.nc;
    return sg;
}

size_t carve_support(Carver &cv, SupportWs &w, const laue_geometry *g, int n_planes, int64_t n_obs,
                     const SupportGrid &sg) {
    const int nb = g->n_rot * g->n_det;
    const int64_t cells = static_cast<int64_t>(nb) * sg.nc * sg.nc;
    w.ooff = cv.take<int64_t>(nb + 1);
    w.probe = cv.take<int>(std::max(n_planes, 1));
    w.cnt = cv.take<int>(cells);
    w.cell_of = cv.take<int>(std::max<int64_t>(n_obs, 1));
    w.coff = cv.take<int64_t>(cells + 1);
    w.pts = cv.take<float2>(std::max<int64_t>(n_obs, 1));
    return cv.size();
}

struct SelectWs {
    SelState *st;
    uint32_t *hist;
    int *flag;
    int64_t *scan;
};

size_t carve_select(Carver &cv, SelectWs &w, int64_t n) {
    w.st = cv.take<SelState>(1);
    w.hist = cv.take<uint32_t>(256);
    w.flag = cv.take<int>(std::max<int64_t>(n, 1));
    w.scan = cv.take<int64_t>(n + 1);
    return cv.size();
}

bool support_params_ok(const laue_support_params *p) {
    return p && std::isfinite(p->radius_mm) && p->radius_mm > 0 && p->n_support_planes >= 0;
}

}  // namespace
}  // namespace laue

using namespace laue;

extern "C" size_t laue_candidate_support_workspace_size(const laue_geometry *geom, int32_t n_planes,
                                                        int64_t n_obs, const laue_support_params *par) {
    if (!geom || validate_geometry(geom) != LAUE_OK || n_planes < 0 || n_obs < 0 || !support_params_ok(par))
        return 0;
    Carver cv(nullptr);
    SupportWs w;
    return carve_support(cv, w, geom, n_planes, n_obs, make_grid(geom, par->radius_mm));
}

extern "C" int laue_candidate_support(const laue_geometry *geom, const laue_planes *planes,
                                      const laue_obs_spots *obs, const laue_candidates *cand,
                                      const laue_support_params *par, void *ws, size_t ws_bytes,
                                      void *stream) {
    clear_error();
    int rc;
    if ((rc = validate_geometry(geom)) || (rc = validate_planes(planes))) return rc;
    LAUE_REQUIRE(support_params_ok(par), LAUE_EINVAL, "bad support parameters");
    LAUE_REQUIRE(obs && obs->block_off && obs->n >= 0 && (obs->n == 0 || (obs->p1 && obs->p2)), LAUE_EINVAL,
                 "detected spots are NULL");
    LAUE_REQUIRE(obs->n < (int64_t(1) << 31), LAUE_EINVAL, "too many detected spots");
    LAUE_REQUIRE(cand && cand->n >= 0 && (cand->n == 0 || (cand->q && cand->spot_a && cand->feat)),
                 LAUE_EINVAL, "candidates need q, spot_a and feat");
    const int nb = geom->n_rot * geom->n_det;
    LAUE_REQUIRE(obs->block_off[0] == 0 && obs->block_off[nb] == obs->n, LAUE_EINVAL,
                 "detected-spot block offsets must run from 0 to n");
    for (int b = 0; b < nb; ++b)
        LAUE_REQUIRE(obs->block_off[b + 1] >= obs->block_off[b], LAUE_EINVAL,
                     "detected-spot block offsets must be non-decreasing");
    hipStream_t s = static_cast<hipStream_t>(stream);
    const SupportGrid sg = make_grid(geom, par->radius_mm);
    Carver cv(ws);
    SupportWs w;
    const size_t need = carve_support(cv, w, geom, planes->n, obs->n, sg);
    if ((rc = check_ws(ws, ws_bytes, need))) return rc;
    if (cand->n == 0) return LAUE_OK;
    // probe planes: the first n_support_planes planes without a lower-order parallel plane
    const int M = planes->n, Mp = std::min(M, par->n_support_planes);
    std::vector<int> hp(M), probe;
    LAUE_CHECK_HIP(hipMemcpyAsync(hp.data(), planes->harmonic_prev, M * sizeof(int), hipMemcpyDeviceToHost, s));
    LAUE_CHECK_HIP(hipStreamSynchronize(s));
    for (int m = 0; m < Mp; ++m)
        if (hp[m] < 0) probe.push_back(m);
    if (!probe.empty())
        LAUE_CHECK_HIP(hipMemcpyAsync(w.probe, probe.data(), probe.size() * sizeof(int), hipMemcpyHostToDevice, s));
    LAUE_CHECK_HIP(hipMemcpyAsync(w.ooff, obs->block_off, (nb + 1) * sizeof(int64_t), hipMemcpyHostToDevice, s));
    const int64_t cells = static_cast<int64_t>(nb) * sg.nc * sg.nc;
    LAUE_CHECK_HIP(hipMemsetAsync(w.cnt, 0, cells * sizeof(int), s));
    if (obs->n > 0) {
        const unsigned gb = static_cast<unsigned>((obs->n + 255) / 256);
        k_grid_count<<<gb, 256, 0, s>>>(obs->p1, obs->p2, w.ooff, nb, obs->n, sg, w.cnt, w.cell_of);
        LAUE_CHECK_HIP(hipGetLastError());
    }
    if ((rc = launch_scan(w.cnt, w.coff, cells, s))) return rc;
    LAUE_CHECK_HIP(hipMemsetAsync(w.cnt, 0, cells * sizeof(int), s));
    if (obs->n > 0) {
        const unsigned gb = static_cast<unsigned>((obs->n + 255) / 256);
        k_grid_fill<<<gb, 256, 0, s>>>(obs->p1, obs->p2, obs->n, w.cell_of, w.coff, w.cnt, w.pts);
        LAUE_CHECK_HIP(hipGetLastError());
    }
    k_support<<<static_cast<unsigned>((cand->n + 127) / 128), 128, 0, s>>>(
        *geom, planes->w, planes->d, w.probe, static_cast<int>(probe.size()), cand->q, cand->spot_a, cand->n,
        w.ooff, obs->n, sg, w.coff, w.pts, par->radius_mm, cand->feat);
    LAUE_CHECK_HIP(hipGetLastError());
    return LAUE_OK;
}

extern "C" int laue_candidate_labels(const laue_candidates *cand, const int32_t *spot_grain, int64_t n_obs,
                                     const laue_grains *truth, double max_deg, float *label, float *mis_deg,
                                     void *stream) {
    clear_error();
    int rc;
    LAUE_REQUIRE(cand && cand->n >= 0 && label, LAUE_EINVAL, "NULL argument");
    if ((rc = validate_grains(truth))) return rc;
    LAUE_REQUIRE(cand->n == 0 || (cand->q && cand->spot_a && cand->spot_b && spot_grain), LAUE_EINVAL,
                 "candidates need q, spot_a and spot_b");
    LAUE_REQUIRE(std::isfinite(max_deg) && max_deg >= 0 && max_deg <= 180, LAUE_EINVAL, "bad angle");
    if (cand->n == 0) return LAUE_OK;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const double ch = std::cos(0.5 * max_deg * M_PI / 180.0);
    k_labels<<<static_cast<unsigned>((cand->n + 255) / 256), 256, 0, s>>>(
        cand->q, cand->spot_a, cand->spot_b, cand->n, spot_grain, n_obs, truth->q, truth->n, ch, label, mis_deg);
    LAUE_CHECK_HIP(hipGetLastError());
    return LAUE_OK;
}

extern "C" int laue_candidate_labels_nearest(const laue_candidates *cand, const laue_grains *truth,
                                             double max_deg, float *label, float *mis_deg, int32_t *nearest,
                                             void *stream) {
    clear_error();
    int rc;
    LAUE_REQUIRE(cand && cand->n >= 0 && label, LAUE_EINVAL, "NULL argument");
    if ((rc = validate_grains(truth))) return rc;
    LAUE_REQUIRE(cand->n == 0 || cand->q, LAUE_EINVAL, "candidates need q");
    LAUE_REQUIRE(std::isfinite(max_deg) && max_deg >= 0 && max_deg <= 180, LAUE_EINVAL, "bad angle");
    if (cand->n == 0) return LAUE_OK;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const double ch = std::cos(0.5 * max_deg * M_PI / 180.0);
    k_labels_nearest<<<static_cast<unsigned>((cand->n + 255) / 256), 256, 0, s>>>(
        cand->q, cand->n, truth->q, truth->n, ch, label, mis_deg, nearest);
    LAUE_CHECK_HIP(hipGetLastError());
    return LAUE_OK;
}

extern "C" size_t laue_pairs_same_grain_workspace_size(const laue_geometry *geom) {
    if (!geom || validate_geometry(geom) != LAUE_OK) return 0;
    Carver cv(nullptr);
    cv.take<int64_t>(geom->n_rot * geom->n_det + 1);
    return cv.size();
}

extern "C" int laue_pairs_same_grain(const laue_geometry *geom, const laue_obs_spots *obs,
                                     const int32_t *spot_grain, int64_t n_pairs, uint64_t seed, int32_t *out_a,
                                     int32_t *out_b, void *ws, size_t ws_bytes, void *stream) {
    clear_error();
    int rc;
    if ((rc = validate_geometry(geom))) return rc;
    const int nb = geom->n_rot * geom->n_det;
    LAUE_REQUIRE(obs && obs->block_off && obs->n >= 0 && obs->n < (int64_t(1) << 31), LAUE_EINVAL,
                 "bad detected spots");
    LAUE_REQUIRE(obs->block_off[0] == 0 && obs->block_off[nb] == obs->n, LAUE_EINVAL,
                 "detected-spot block offsets must run from 0 to n");
    for (int b = 0; b < nb; ++b)
        LAUE_REQUIRE(obs->block_off[b + 1] >= obs->block_off[b], LAUE_EINVAL,
                     "detected-spot block offsets must be non-decreasing");
    LAUE_REQUIRE(n_pairs >= 0 && n_pairs < (int64_t(1) << 31), LAUE_EINVAL, "bad n_pairs");
    LAUE_REQUIRE(n_pairs == 0 || (out_a && out_b && (obs->n == 0 || spot_grain)), LAUE_EINVAL, "NULL argument");
    hipStream_t s = static_cast<hipStream_t>(stream);
    Carver cv(ws);
    int64_t *ooff = cv.take<int64_t>(nb + 1);
    if ((rc = check_ws(ws, ws_bytes, cv.size()))) return rc;
    if (n_pairs == 0) return LAUE_OK;
    LAUE_CHECK_HIP(hipMemcpyAsync(ooff, obs->block_off, (nb + 1) * sizeof(int64_t), hipMemcpyHostToDevice, s));
    k_same_pairs<<<static_cast<unsigned>((n_pairs + 255) / 256), 256, 0, s>>>(
        ooff, geom->n_rot, geom->n_det, spot_grain, obs->n, n_pairs, static_cast<uint32_t>(seed & 0xffffffffu),
        static_cast<uint32_t>(seed >> 32), out_a, out_b);
    LAUE_CHECK_HIP(hipGetLastError());
    return LAUE_OK;
}

extern "C" size_t laue_select_top_workspace_size(int64_t n) {
    if (n < 0) return 0;
    Carver cv(nullptr);
    SelectWs w;
    return carve_select(cv, w, n);
}

extern "C" int laue_select_top(const float *score, int64_t n, int64_t k, int32_t *out, void *ws,
                               size_t ws_bytes, void *stream) {
    clear_error();
    int rc;
    LAUE_REQUIRE(n >= 0 && n < (int64_t(1) << 31) && k >= 0 && k <= n, LAUE_EINVAL, "need 0 <= k <= n < 2^31");
    LAUE_REQUIRE(k == 0 || (score && out), LAUE_EINVAL, "NULL argument");
    hipStream_t s = static_cast<hipStream_t>(stream);
    Carver cv(ws);
    SelectWs w;
    const size_t need = carve_select(cv, w, n);
    if ((rc = check_ws(ws, ws_bytes, need))) return rc;
    if (k == 0) return LAUE_OK;
    const unsigned g1 = static_cast<unsigned>((n + 255) / 256);
    const unsigned gh = std::min<unsigned>(g1, 2048u);
    k_sel_init<<<1, 1, 0, s>>>(w.st, k, w.hist);
    for (int shift = 24; shift >= 0; shift -= 8) {
        k_sel_hist<<<gh, 256, 0, s>>>(score, n, w.st, shift, w.hist);
        k_sel_pick<<<1, 1, 0, s>>>(w.st, shift, w.hist);
    }
    k_sel_eq<<<g1, 256, 0, s>>>(score, n, w.st, w.flag);
    LAUE_CHECK_HIP(hipGetLastError());
    if ((rc = launch_scan(w.flag, w.scan, n, s))) return rc;
    k_sel_take<<<g1, 256, 0, s>>>(score, n, w.st, w.scan, w.flag);
    LAUE_CHECK_HIP(hipGetLastError());
    if ((rc = launch_scan(w.flag, w.scan, n, s))) return rc;
    k_sel_write<<<g1, 256, 0, s>>>(w.flag, w.scan, n, k, out);
    LAUE_CHECK_HIP(hipGetLastError());
    return LAUE_OK;
}
