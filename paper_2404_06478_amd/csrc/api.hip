// Host-side helpers of liblaueot: errors, geometry validation, plane lists.
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <numeric>
#include <tuple>

#include "common.h"

namespace laue {

static thread_local std::string g_err;

void set_error(const std::string &msg) { g_err = msg; }
void clear_error() { g_err.clear(); }

bool log_enabled() {
    static const bool on = [] {
        const char *v = std::getenv("LAUE_LOG");
        return v != nullptr && v[0] != '\0' && std::strcmp(v, "0") != 0;
    }();
    return on;
}

void log_line(const char *fmt, ...) {
    if (!log_enabled()) return;
    std::va_list ap;
    va_start(ap, fmt);
    std::fputs("liblaueot: ", stderr);
    std::vfprintf(stderr, fmt, ap);
    std::fputc('\n', stderr);
    std::fflush(stderr);
    va_end(ap);
}

int check_ws(void *ws, size_t ws_bytes, size_t need) {
    if (need == 0) return LAUE_OK;
    if (ws == nullptr || ws_bytes < need) {
        set_error("workspace too small: need " + std::to_string(need) + " bytes, got " +
                  std::to_string(ws_bytes));
        return LAUE_EWORKSPACE;
    }
    if ((reinterpret_cast<uintptr_t>(ws) & 255) != 0) {
        set_error("workspace must be 256-byte aligned");
        return LAUE_EWORKSPACE;
    }
    return LAUE_OK;
}

static bool finite3(const double *v) {
    return std::isfinite(v[0]) && std::isfinite(v[1]) && std::isfinite(v[2]);
}

int validate_geometry(const laue_geometry *g) {
    LAUE_REQUIRE(g != nullptr, LAUE_EINVAL, "geometry is NULL");
    LAUE_REQUIRE(g->n_rot >= 1 && g->n_rot <= LAUE_MAX_ROT, LAUE_EINVAL, "n_rot out of range");
    LAUE_REQUIRE(g->n_det >= 1 && g->n_det <= LAUE_MAX_DET, LAUE_EINVAL, "n_det out of range");
    LAUE_REQUIRE(std::isfinite(g->omega0) && std::isfinite(g->domega), LAUE_EINVAL,
                 "rotation angles must be finite");
    LAUE_REQUIRE(std::isfinite(g->lambda_min) && std::isfinite(g->lambda_max) &&
                     g->lambda_min > 0 && g->lambda_max >= g->lambda_min,
                 LAUE_EINVAL, "bad wavelength band");
    for (int d = 0; d < g->n_det; ++d) {
        const laue_detector &D = g->det[d];
        LAUE_REQUIRE(finite3(D.center) && finite3(D.normal) && finite3(D.axis1) &&
                         finite3(D.axis2) && std::isfinite(D.half_size) && D.half_size > 0,
                     LAUE_EINVAL, "bad detector");
    }
    return LAUE_OK;
}

void make_geomf(const laue_geometry *g, GeomF *o) {
    std::memset(o, 0, sizeof(GeomF));
    o->n_rot = g->n_rot;
    o->n_det = g->n_det;
    o->lam_min = static_cast<float>(g->lambda_min);
    o->lam_max = static_cast<float>(g->lambda_max);
    for (int d = 0; d < g->n_det; ++d) {
        const laue_detector &D = g->det[d];
        for (int k = 0; k < 3; ++k) {
            o->det[d].c[k] = static_cast<float>(D.center[k]);
            o->det[d].n[k] = static_cast<float>(D.normal[k]);
            o->det[d].a1[k] = static_cast<float>(D.axis1[k]);
            o->det[d].a2[k] = static_cast<float>(D.axis2[k]);
        }
        o->det[d].half = static_cast<float>(D.half_size);
    }
    for (int t = 0; t < g->n_rot; ++t) {
        double om = g->omega0 + g->domega * t;
        o->cs[t][0] = static_cast<float>(std::cos(om));
        o->cs[t][1] = static_cast<float>(std::sin(om));
    }
}

}  // namespace laue

using namespace laue;

extern "C" int laue_version(void) { return 200; }

extern "C" const char *laue_last_error(void) { return g_err.c_str(); }

static bool allowed(int h, int k, int l, char c) {
    if (c == 'P') return true;
    if (c == 'I') return ((h + k + l) % 2 + 2) % 2 == 0;
    int ph = ((h % 2) + 2) % 2, pk = ((k % 2) + 2) % 2, pl = ((l % 2) + 2) % 2;
    return ph == pk && pk == pl;
}

static int gcd3(int a, int b, int c) { return std::gcd(std::gcd(std::abs(a), std::abs(b)), std::abs(c)); }

extern "C" int laue_ot_defaults(double sigma_mm, double distance, int64_t n_model, laue_ot_params *out) {
    clear_error();
    LAUE_REQUIRE(out != nullptr, LAUE_EINVAL, "output is NULL");
    LAUE_REQUIRE(std::isfinite(sigma_mm) && sigma_mm > 0 && std::isfinite(distance) && distance > 0 && n_model >= 0,
                 LAUE_EINVAL, "sigma_mm and distance must be > 0 and n_model >= 0");
    *out = laue_ot_params{};
    out->eps = 2.0 * sigma_mm * sigma_mm;
    out->distance = distance;
    out->c_out = 2.0 * distance * distance * (1.0 - std::cos(3.0 * sigma_mm / distance));
    out->c_unm = 0.0;
    out->c_sink = out->c_out;
    out->t_b = std::ceil(0.4 * static_cast<double>(n_model));
    out->tol = 1e-5;
    out->n_max = 2000;
    return LAUE_OK;
}

extern "C" int laue_planes_cubic(double a, char centering, int n_max, int32_t *n_planes,
                                 int32_t *hkl, float *w, float *d, int32_t *harmonic_prev) {
    clear_error();
    LAUE_REQUIRE(n_planes != nullptr, LAUE_EINVAL, "n_planes is NULL");
    LAUE_REQUIRE(centering == 'P' || centering == 'I' || centering == 'F', LAUE_EINVAL,
                 "centering must be 'P', 'I' or 'F'");
    LAUE_REQUIRE(n_max >= 1 && n_max <= 4096, LAUE_EINVAL, "n_max out of range");
    LAUE_REQUIRE(std::isfinite(a) && a > 0, LAUE_EINVAL, "lattice constant must be positive");
    std::vector<std::tuple<int, int, int, int>> rows;
    int lim = static_cast<int>(std::sqrt(static_cast<double>(n_max))) + 1;
    for (int h = -lim; h <= lim; ++h)
        for (int k = -lim; k <= lim; ++k)
            for (int l = -lim; l <= lim; ++l) {
                int n = h * h + k * k + l * l;
                if (n == 0 || n > n_max || !allowed(h, k, l, centering)) continue;
                rows.emplace_back(n, h, k, l);
            }
    std::sort(rows.begin(), rows.end());
    *n_planes = static_cast<int32_t>(rows.size());
    if (hkl == nullptr && w == nullptr && d == nullptr && harmonic_prev == nullptr) return LAUE_OK;
    std::map<std::tuple<int, int, int>, int> index;
    for (size_t i = 0; i < rows.size(); ++i)
        index[{std::get<1>(rows[i]), std::get<2>(rows[i]), std::get<3>(rows[i])}] = static_cast<int>(i);
    for (size_t i = 0; i < rows.size(); ++i) {
        auto [n, h, k, l] = rows[i];
        double sq = std::sqrt(static_cast<double>(n));
        if (hkl) {
            hkl[3 * i] = h;
            hkl[3 * i + 1] = k;
            hkl[3 * i + 2] = l;
        }
        if (w) {
            w[3 * i] = static_cast<float>(h / sq);
            w[3 * i + 1] = static_cast<float>(k / sq);
            w[3 * i + 2] = static_cast<float>(l / sq);
        }
        if (d) d[i] = static_cast<float>(a / sq);
        if (harmonic_prev) {
            int g = gcd3(h, k, l), p = -1;
            for (int mult = g - 1; mult >= 1 && p < 0; --mult) {
                auto it = index.find({h / g * mult, k / g * mult, l / g * mult});
                if (it != index.end()) p = it->second;
            }
            harmonic_prev[i] = p;
        }
    }
    return LAUE_OK;
}
