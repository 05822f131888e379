// Sobol-grid starts of single-grain fitting (Sec. 6.1): Sobol points in the
// six-dimensional (R, x) space, orientations as modified Rodrigues parameters
// restricted to the cubic fundamental zone, positions within the sample box.
//
// Point n, coordinate d: XOR of the direction numbers V_d[k] over the bits k
// of the Gray code n ^ (n >> 1), over 2^32 (Sobol's sequence in the
// Antonov-Saleev order; Joe and Kuo's primitive polynomials and initial
// numbers for dimensions 2..6).  One thread per point flags whether its
// orientation lies in the zone; a stable device select keeps the flagged
// indices in order; a second pass writes their (q, x).
#include <algorithm>
#include <cmath>

#include <hipcub/hipcub.hpp>

#include "common.h"

namespace laue {
namespace {

constexpr int kSobolDims = 6;
constexpr int kSobolBits = 32;

struct SobolArgs {
    uint32_t V[kSobolDims][kSobolBits];
    double mrp_half;      // half side of the MRP cube
    double x_half[3];     // half extents of the position box (mm)
    double r_face;        // tan(pi / 8): the zone's faces along the cube axes
    int restrict_fz;
};

// Direction numbers: dimension 1 is the van der Corput sequence; 2..6 take the
// degree s, coefficient bits a and initial m_1..m_s of Joe and Kuo's table,
// extended by V[k] = V[k-s] ^ (V[k-s] >> s) ^ XOR_{i<s, a_i} V[k-i].
void sobol_directions(SobolArgs &A) {
    struct Poly {
        int s, a, m[4];
    };
    static const Poly tab[kSobolDims - 1] = {
        {1, 0, {1, 0, 0, 0}}, {2, 1, {1, 3, 0, 0}}, {3, 1, {1, 3, 1, 0}}, {3, 2, {1, 1, 1, 0}}, {4, 1, {1, 1, 3, 3}}};
    for (int k = 0; k < kSobolBits; ++k) A.V[0][k] = 1u << (kSobolBits - 1 - k);
    for (int d = 1; d < kSobolDims; ++d) {
        const Poly &P = tab[d - 1];
        uint32_t V[kSobolBits + 1] = {};
        for (int k = 1; k <= P.s; ++k) V[k] = static_cast<uint32_t>(P.m[k - 1]) << (kSobolBits - k);
        for (int k = P.s + 1; k <= kSobolBits; ++k) {
            uint32_t v = V[k - P.s] ^ (V[k - P.s] >> P.s);
            for (int i = 1; i < P.s; ++i)
                if ((P.a >> (P.s - 1 - i)) & 1) v ^= V[k - i];
            V[k] = v;
        }
        for (int k = 0; k < kSobolBits; ++k) A.V[d][k] = V[k + 1];
    }
}

// The start of Sobol point idx: unit quaternion q (q0 > 0) and position x;
// returns whether the orientation lies in the cubic fundamental zone.  The
// FP64 operations are kept separate (no contraction) so that the zone test
// rounds as a plain evaluation of the same formulas does.
__device__ bool sobol_start(const SobolArgs &A, int64_t idx, double *q, double *x) {
#pragma clang fp contract(off)
    const uint64_t g = static_cast<uint64_t>(idx) ^ (static_cast<uint64_t>(idx) >> 1);
    double u[kSobolDims];
    for (int d = 0; d < kSobolDims; ++d) {
        uint32_t v = 0;
        for (int k = 0; k < kSobolBits; ++k)
            if ((g >> k) & 1u) v ^= A.V[d][k];
        u[d] = static_cast<double>(v) / 4294967296.0;
    }
    double p[3];
    for (int k = 0; k < 3; ++k) p[k] = (2.0 * u[k] - 1.0) * A.mrp_half;
    const double s = p[0] * p[0] + p[1] * p[1] + p[2] * p[2];
    q[0] = (1.0 - s) / (1.0 + s);
    for (int k = 0; k < 3; ++k) q[1 + k] = (2.0 * p[k]) / (1.0 + s);
    for (int k = 0; k < 3; ++k) x[k] = (2.0 * u[3 + k] - 1.0) * A.x_half[k];
    if (!A.restrict_fz) return true;
    const double r0 = fabs(q[1] / q[0]), r1 = fabs(q[2] / q[0]), r2 = fabs(q[3] / q[0]);
    return r0 <= A.r_face && r1 <= A.r_face && r2 <= A.r_face && (r0 + r1) + r2 <= 1.0;
}

__global__ void k_sobol_flags(const SobolArgs A, int64_t first, int64_t n, uint8_t *__restrict__ flag) {
    const int64_t r = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (r >= n) return;
    double q[4], x[3];
    flag[r] = sobol_start(A, first + r, q, x) ? 1 : 0;
}

__global__ void k_sobol_gather(const SobolArgs A, int64_t first, const int *__restrict__ sel,
                               const int *__restrict__ count, double *__restrict__ oq, double *__restrict__ ox) {
    const int64_t r = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (r >= *count) return;
    double q[4], x[3];
    sobol_start(A, first + sel[r], q, x);
    for (int k = 0; k < 4; ++k) oq[4 * r + k] = q[k];
    for (int k = 0; k < 3; ++k) ox[3 * r + k] = x[k];
}

struct SobolWs {
    uint8_t *flag;
    int *sel;
    int *count;
    void *tmp;
    size_t tmp_bytes;
};

size_t select_tmp_bytes(int64_t n) {
    size_t b = 0;
    hipcub::CountingInputIterator<int> it(0);
    if (hipcub::DeviceSelect::Flagged(nullptr, b, it, static_cast<uint8_t *>(nullptr), static_cast<int *>(nullptr),
                                      static_cast<int *>(nullptr), static_cast<int>(n)) != hipSuccess)
        return 0;
    return b;
}

size_t carve_sobol(Carver &cv, SobolWs &w, int64_t n) {
    const int64_t m = std::max<int64_t>(n, 1);
    w.flag = cv.take<uint8_t>(m);
    w.sel = cv.take<int>(m);
    w.count = cv.take<int>(1);
    w.tmp_bytes = select_tmp_bytes(m) + 256;
    w.tmp = cv.take<char>(w.tmp_bytes);
    return cv.size();
}

int validate_sobol(const laue_sobol_params *p, int64_t n) {
    LAUE_REQUIRE(p != nullptr, LAUE_EINVAL, "Sobol parameters are NULL");
    LAUE_REQUIRE(n >= 0 && n < (int64_t(1) << 31), LAUE_EINVAL, "n_points must be in [0, 2^31)");
    LAUE_REQUIRE(p->first >= 0 && p->first + n < (int64_t(1) << 32), LAUE_EINVAL,
                 "Sobol indices must stay below 2^32");
    LAUE_REQUIRE(std::isfinite(p->mrp_half) && p->mrp_half >= 0 && p->mrp_half <= 1.0, LAUE_EINVAL,
                 "mrp_half must be in [0, 1] (0: the cubic zone's bound)");
    for (int k = 0; k < 3; ++k)
        LAUE_REQUIRE(std::isfinite(p->x_half[k]) && p->x_half[k] >= 0, LAUE_EINVAL, "x_half must be >= 0");
    return LAUE_OK;
}

}  // namespace

size_t sobol_workspace_size(int64_t n) {
    Carver cv(nullptr);
    SobolWs w;
    return carve_sobol(cv, w, n);
}

int sobol_starts(const laue_sobol_params *par, int64_t n, double *q, double *x, int64_t *n_kept, void *ws,
                 size_t ws_bytes, hipStream_t s) {
    int rc;
    if ((rc = validate_sobol(par, n))) return rc;
    LAUE_REQUIRE(n_kept != nullptr, LAUE_EINVAL, "n_kept is NULL");
    LAUE_REQUIRE(n == 0 || (q && x), LAUE_EINVAL, "q or x is NULL");
    *n_kept = 0;
    if (n == 0) return LAUE_OK;
    Carver cv(ws);
    SobolWs w;
    const size_t need = carve_sobol(cv, w, n);
    if ((rc = check_ws(ws, ws_bytes, need))) return rc;
    LAUE_REQUIRE(w.tmp_bytes > 256, LAUE_EDEVICE, "device select sizing failed");
    SobolArgs A;
    sobol_directions(A);
    A.mrp_half = par->mrp_half > 0 ? par->mrp_half : std::tan(M_PI / 16.0);
    for (int k = 0; k < 3; ++k) A.x_half[k] = par->x_half[k];
    A.r_face = std::tan(M_PI / 8.0);
    A.restrict_fz = par->restrict_fz ? 1 : 0;
    const unsigned nb = static_cast<unsigned>((n + 255) / 256);
    k_sobol_flags<<<nb, 256, 0, s>>>(A, par->first, n, w.flag);
    LAUE_CHECK_HIP(hipGetLastError());
    hipcub::CountingInputIterator<int> it(0);
    size_t tb = w.tmp_bytes;
    LAUE_CHECK_HIP(hipcub::DeviceSelect::Flagged(w.tmp, tb, it, w.flag, w.sel, w.count, static_cast<int>(n), s));
    k_sobol_gather<<<nb, 256, 0, s>>>(A, par->first, w.sel, w.count, q, x);
    LAUE_CHECK_HIP(hipGetLastError());
    int cnt = 0;
    LAUE_CHECK_HIP(hipMemcpyAsync(&cnt, w.count, sizeof(int), hipMemcpyDeviceToHost, s));
    LAUE_CHECK_HIP(hipStreamSynchronize(s));
    *n_kept = cnt;
    return LAUE_OK;
}

}  // namespace laue

using namespace laue;

extern "C" size_t laue_sobol_workspace_size(int64_t n_points) {
    if (n_points < 0) return 0;
    return sobol_workspace_size(n_points);
}

extern "C" int laue_sobol_starts(const laue_sobol_params *par, int64_t n_points, double *q, double *x,
                                 int64_t *n_kept, void *ws, size_t ws_bytes, void *stream) {
    clear_error();
    return sobol_starts(par, n_points, q, x, n_kept, ws, ws_bytes, static_cast<hipStream_t>(stream));
}
