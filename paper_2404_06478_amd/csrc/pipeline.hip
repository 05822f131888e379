// End-to-end indexing (the multigrain solve of Sec. 6 and Alg. MultiGrainLaueOT
// with spot-pair candidates in place of the orientation grid, or with the
// Sobol-grid starts of Sec. 6.1):
//   candidates -> [learned: support features, network, top fraction] ->
//   single-grain refinement and scoring -> greedy SPOT -> k* prototypes ->
//   model spots of the prototypes (frozen) -> EM with annealed entropic OT.
// Every stage is one of the library's entry points; this file only carves the
// caller's workspace and moves indices between them.  The stages are
// synchronous, and their wall-clock times (host clock around each stage,
// stream synchronised) are reported.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <vector>

#include "common.h"

namespace laue {
namespace {

struct IndexWs {
    // candidates
    double *cq;
    int *pair, *ma, *mb, *sa, *sb;
    float *feat, *prob;
    int *sel;
    // scored subset (refined in place)
    double *gq, *gx;
    int *n_model, *n_unm;
    uint8_t *keep;
    int64_t *loff;
    int *lrow;
    float *lval;
    int *picks;
    double *gains;
    // model spots and potentials of the EM
    int *mplane, *mgrain, *mblock;
    float *s1, *s2, *vn, *v1, *v2, *lam;
    uint8_t *flags;
    float *f, *g;
    void *scratch;
    size_t scratch_bytes;
};

int64_t n_scored_max(const laue_index_params *p) {
    if (p->mode == LAUE_INDEX_LEARNED)
        return std::min<int64_t>(p->max_candidates,
                                 static_cast<int64_t>(std::ceil(p->top_frac * static_cast<double>(p->max_candidates))));
    return p->max_candidates;
}

size_t scratch_size(const laue_geometry *g, int n_planes, int64_t n_obs, const laue_index_params *p) {
    size_t s = laue_candidates_workspace_size(g, n_planes, p->cand.n_pairs);
    if (p->mode == LAUE_INDEX_LEARNED) {
        s = std::max(s, laue_candidate_support_workspace_size(g, n_planes, n_obs, &p->support));
        s = std::max(s, laue_mlp_forward_workspace_size(p->max_candidates));
        s = std::max(s, laue_select_top_workspace_size(p->max_candidates));
    }
    if (p->mode == LAUE_INDEX_SOBOL) s = std::max(s, laue_sobol_workspace_size(p->max_candidates));
    s = std::max(s, laue_score_workspace_size(g, n_obs, &p->score));
    s = std::max(s, laue_spot_greedy_workspace_size(static_cast<int32_t>(n_scored_max(p)), n_obs));
    s = std::max(s, laue_forward_workspace_size(g, n_planes, p->k_max));
    s = std::max(s, laue_sinkhorn_workspace_size(g, n_obs, p->max_model_spots, p->k_max));
    if (p->em.ot.rho > 0 || (p->em.eps_cool > 0.0 && !(p->em.eps_start > 0.0))) {
        const int64_t no = n_obs, nm = p->max_model_spots;
        const int32_t ng = p->k_max;
        s = std::max(s, laue_sparse_workspace_size(1, g, &no, &nm, &ng, p->em.ot.rho > 0 ? p->em.ot.rho : 32));
    }
    return s;
}

size_t carve_index(Carver &cv, IndexWs &w, const laue_geometry *g, int n_planes, int64_t n_obs,
                   const laue_index_params *p) {
    const int64_t C = std::max<int64_t>(p->max_candidates, 1), S = std::max<int64_t>(n_scored_max(p), 1);
    const int64_t J = std::max<int64_t>(p->max_model_spots, 1), K = std::max(p->k_max, 1);
    const bool learned = p->mode == LAUE_INDEX_LEARNED;
    w.cq = cv.take<double>(4 * C);
    w.pair = cv.take<int>(C);
    w.ma = cv.take<int>(C);
    w.mb = cv.take<int>(C);
    w.sa = cv.take<int>(C);
    w.sb = cv.take<int>(C);
    w.feat = learned ? cv.take<float>(16 * C) : nullptr;
    w.prob = learned ? cv.take<float>(C) : nullptr;
    w.sel = learned ? cv.take<int>(S) : nullptr;
    w.gq = cv.take<double>(4 * S);
    w.gx = cv.take<double>(3 * S);
    w.n_model = cv.take<int>(S);
    w.n_unm = cv.take<int>(S);
    w.keep = cv.take<uint8_t>(S);
    w.loff = cv.take<int64_t>(S + 1);
    w.lrow = cv.take<int>(std::max<int64_t>(p->lbar_cap, 1));
    w.lval = cv.take<float>(std::max<int64_t>(p->lbar_cap, 1));
    w.picks = cv.take<int>(K);
    w.gains = cv.take<double>(K);
    w.mplane = cv.take<int>(J);
    w.mgrain = cv.take<int>(J);
    w.mblock = cv.take<int>(J);
    w.s1 = cv.take<float>(J);
    w.s2 = cv.take<float>(J);
    w.vn = cv.take<float>(J);
    w.v1 = cv.take<float>(J);
    w.v2 = cv.take<float>(J);
    w.lam = cv.take<float>(J);
    w.flags = cv.take<uint8_t>(J);
    w.f = cv.take<float>(std::max<int64_t>(n_obs, 1));
    w.g = cv.take<float>(J);
    w.scratch_bytes = scratch_size(g, n_planes, n_obs, p);
    w.scratch = cv.take<char>(w.scratch_bytes);
    return cv.size();
}

// scored grains: q from the candidates (all, or the selected ones), x = 0
__global__ void k_seed_grains(const double *__restrict__ cq, const int *__restrict__ sel, int64_t n,
                              double *__restrict__ gq, double *__restrict__ gx) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int64_t c = sel ? sel[i] : i;
    for (int k = 0; k < 4; ++k) gq[4 * i + k] = cq[4 * c + k];
    for (int k = 0; k < 3; ++k) gx[3 * i + k] = 0.0;
}

__global__ void k_gather_protos(const double *__restrict__ gq, const double *__restrict__ gx,
                                const int *__restrict__ picks, int k, double *__restrict__ oq,
                                double *__restrict__ ox) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= k) return;
    const int c = picks[i];
    for (int j = 0; j < 4; ++j) oq[4 * i + j] = gq[4 * c + j];
    for (int j = 0; j < 3; ++j) ox[3 * i + j] = gx[3 * c + j];
}

__global__ void k_zero_f(float *p, int64_t n) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0.0f;
}

int validate_index_params(const laue_index_params *p) {
    LAUE_REQUIRE(p, LAUE_EINVAL, "NULL index parameters");
    LAUE_REQUIRE(p->mode == LAUE_INDEX_PLAIN || p->mode == LAUE_INDEX_LEARNED || p->mode == LAUE_INDEX_SOBOL,
                 LAUE_EINVAL, "bad index mode");
    LAUE_REQUIRE(p->cand.pair_a == nullptr && p->cand.pair_b == nullptr, LAUE_EINVAL,
                 "indexing draws its own pairs");
    LAUE_REQUIRE(p->max_candidates >= 1 && p->max_candidates < (int64_t(1) << 31), LAUE_EINVAL,
                 "bad candidate capacity");
    LAUE_REQUIRE(p->k_max >= 1 && p->max_model_spots >= 1 && p->lbar_cap >= 1, LAUE_EINVAL, "bad capacities");
    LAUE_REQUIRE(std::isfinite(p->t_b_frac) && p->t_b_frac >= 0 && p->t_b_frac <= 1, LAUE_EINVAL, "bad t_b_frac");
    if (p->mode == LAUE_INDEX_LEARNED) {
        LAUE_REQUIRE(p->mlp != nullptr, LAUE_EINVAL, "learned mode needs a network");
        LAUE_REQUIRE(std::isfinite(p->top_frac) && p->top_frac > 0 && p->top_frac <= 1, LAUE_EINVAL,
                     "bad top fraction");
    }
    return LAUE_OK;
}

// Eq. spot_ngrains: k* where f (the running sum of the greedy's increments)
// bends most, its second difference taken over h picks: argmax over k >= 1 of
// the mean increment of the h picks up to k (m = min(k, h) of them) minus that
// of the h picks after k (increments beyond the picks are 0); lowest k on
// ties.  A step of one pick is the printed difference; the increments of a
// long run of true grains vary by about 1% from pick to pick, so that step can
// peak among the first picks.
constexpr int kPrototypeStep = 8;

int prototype_count(const std::vector<double> &gains, int h) {
    const int K = static_cast<int>(gains.size());
    std::vector<double> f(K + 1, 0.0);
    for (int k = 0; k < K; ++k) f[k + 1] = f[k] + gains[k];
    double best = -INFINITY;
    int arg = K > 0 ? 1 : 0;
    for (int k = 1; k <= K; ++k) {
        const int m = std::min(k, h);
        const double v = (f[k] - f[k - m]) / m - (f[std::min(K, k + h)] - f[k]) / h;
        if (v > best) {
            best = v;
            arg = k;
        }
    }
    return arg;
}

double ms_since(std::chrono::steady_clock::time_point t0) {
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
}

}  // namespace
}  // namespace laue

using namespace laue;

extern "C" size_t laue_index_workspace_size(const laue_geometry *geom, int32_t n_planes, int64_t n_obs,
                                            const laue_index_params *par) {
    if (!geom || validate_geometry(geom) != LAUE_OK || n_planes < 0 || n_obs < 0 || validate_index_params(par))
        return 0;
    Carver cv(nullptr);
    IndexWs w;
    return carve_index(cv, w, geom, n_planes, n_obs, par);
}

namespace laue {
namespace {

// What the EM stage of one sample needs once stages 1-5a have run.
struct EmJob {
    laue_grains protos;
    laue_model_spots model;
    laue_em_params em;
    laue_potentials pot;
    laue_assignments asg;
    bool with_assign;
    std::vector<int64_t> moff;   // host block offsets of model (model.block_off points here)
};

// Stages 1-4 and the first half of 5 for one sample: candidates, proposal,
// refinement and scoring, greedy SPOT, the k* prototypes into out, their
// frozen model spots (w.mplane ... w.flags), the EM's temperatures and bins,
// zeroed potentials (w.f, w.g).  job.protos.n = 0 when k* = 0.
int index_front(const laue_geometry *geom, const laue_planes *planes, const laue_obs_spots *obs,
                const laue_index_params *par, laue_index_out *out, IndexWs &w, laue_index_stats &st, EmJob &job,
                hipStream_t s) {
    int rc;
    void *stream = s;
    const int nb = geom->n_rot * geom->n_det;
    const laue_assignments &as = out->assign;
    job.with_assign = as.j_star && as.grain && as.q_star && as.q_out;
    job.protos = laue_grains{0, out->q, out->x};
    out->n_grains = 0;

    // 1. spot-pair candidates
    auto t0 = std::chrono::steady_clock::now();
    laue_candidates cand{};
    cand.n = par->max_candidates;
    cand.q = w.cq;
    cand.pair = w.pair;
    cand.ma = w.ma;
    cand.mb = w.mb;
    cand.spot_a = w.sa;
    cand.spot_b = w.sb;
    cand.feat = w.feat;
    int64_t n_found = 0;
    const bool sobol = par->mode == LAUE_INDEX_SOBOL;
    if (sobol) {
        // Sobol-grid starts (Sec. 6.1) straight into the scored grains
        if ((rc = laue_sobol_starts(&par->sobol, par->max_candidates, w.gq, w.gx, &n_found, w.scratch,
                                    w.scratch_bytes, stream)))
            return rc;
        cand.n = n_found;
    } else if ((rc = laue_candidates_generate(geom, planes, obs, &par->cand, &cand, &n_found, w.scratch,
                                              w.scratch_bytes, stream))) {
        return rc;
    }
    st.n_candidates = cand.n;
    st.n_candidates_found = n_found;
    st.ms_candidates = ms_since(t0);
    log_line("index: %lld candidates (%lld found) in %.1f ms", static_cast<long long>(cand.n),
             static_cast<long long>(n_found),
             st.ms_candidates);

    // 2. learned proposal: support features, network, top fraction
    int64_t n_sc = cand.n;
    const int *sel = nullptr;
    t0 = std::chrono::steady_clock::now();
    if (par->mode == LAUE_INDEX_LEARNED && cand.n > 0) {
        if ((rc = laue_candidate_support(geom, planes, obs, &cand, &par->support, w.scratch, w.scratch_bytes, stream)))
            return rc;
        if ((rc = laue_mlp_forward(par->mlp, w.feat, cand.n, w.prob, w.scratch, w.scratch_bytes, stream))) return rc;
        n_sc = std::min<int64_t>(cand.n, static_cast<int64_t>(std::ceil(par->top_frac * static_cast<double>(cand.n))));
        if ((rc = laue_select_top(w.prob, cand.n, n_sc, w.sel, w.scratch, w.scratch_bytes, stream))) return rc;
        sel = w.sel;
        LAUE_CHECK_HIP(hipStreamSynchronize(s));
    }
    st.ms_proposal = ms_since(t0);
    st.n_scored = n_sc;
    if (par->mode == LAUE_INDEX_LEARNED)
        log_line("index: proposal kept %lld candidates in %.1f ms", static_cast<long long>(n_sc), st.ms_proposal);

    // 3. single-grain refinement and scoring of the chosen candidates
    t0 = std::chrono::steady_clock::now();
    if (n_sc > 0 && !sobol) {
        k_seed_grains<<<static_cast<unsigned>((n_sc + 255) / 256), 256, 0, s>>>(w.cq, sel, n_sc, w.gq, w.gx);
        LAUE_CHECK_HIP(hipGetLastError());
    }
    laue_grains scored{static_cast<int32_t>(n_sc), w.gq, w.gx};
    laue_score_out so{};
    so.n_model = w.n_model;
    so.n_unmatched = w.n_unm;
    so.keep = w.keep;
    so.lbar_off = w.loff;
    so.lbar_row = w.lrow;
    so.lbar_val = w.lval;
    so.lbar_cap = par->lbar_cap;
    if (n_sc > 0) {
        if ((rc = laue_score_candidates(geom, planes, obs, &scored, &par->score, &so, w.scratch, w.scratch_bytes,
                                        stream)))
            return rc;
    }
    st.lbar_entries = so.lbar_n;
    st.score_pairs = so.pairs_streamed;
    st.score_pairs_evaluated = so.pairs_evaluated;
    st.score_pairs_refine = so.pairs_refine;
    if (log_enabled()) LAUE_CHECK_HIP(hipStreamSynchronize(s));
    st.ms_score = ms_since(t0);
    log_line("index: scored %lld candidates, %lld SPOT entries, in %.1f ms", static_cast<long long>(n_sc),
             static_cast<long long>(so.lbar_n), st.ms_score);

    // 4. greedy SPOT and the number of prototypes k* = argmax_k (D_k - D_{k+1})
    t0 = std::chrono::steady_clock::now();
    int32_t n_picked = 0;
    if (n_sc > 0) {
        const double phi = -par->score.c_out / (2.0 * par->score.sigma_mm * par->score.sigma_mm);
        // the SPOT matrix is not read after the selection: compacted in place
        if ((rc = spot_greedy_inplace(w.loff, w.lrow, w.lval, static_cast<int32_t>(n_sc), obs->n, phi, par->k_max,
                                   w.picks, w.gains, &n_picked, w.scratch, w.scratch_bytes, stream)))
            return rc;
    }
    int k_star = 0;
    if (n_picked > 0) {
        std::vector<double> gains(n_picked);
        LAUE_CHECK_HIP(hipMemcpyAsync(gains.data(), w.gains, n_picked * sizeof(double), hipMemcpyDeviceToHost, s));
        LAUE_CHECK_HIP(hipStreamSynchronize(s));
        k_star = prototype_count(gains, kPrototypeStep);
        k_gather_protos<<<(k_star + 63) / 64, 64, 0, s>>>(w.gq, w.gx, w.picks, k_star, out->q, out->x);
        LAUE_CHECK_HIP(hipGetLastError());
    }
    st.n_picked = n_picked;
    st.n_prototypes = k_star;
    st.ms_greedy = ms_since(t0);
    log_line("index: greedy picked %d, k* = %d, in %.1f ms", n_picked, k_star, st.ms_greedy);
    out->n_grains = k_star;
    if (k_star == 0) {
        LAUE_CHECK_HIP(hipStreamSynchronize(s));
        return LAUE_OK;
    }

    // 5. frozen model spots of the prototypes, then (the caller) EM
    t0 = std::chrono::steady_clock::now();
    laue_grains protos{k_star, out->q, out->x};
    job.moff.assign(nb + 1, 0);
    laue_model_spots model{};
    model.n = par->max_model_spots;
    model.plane = w.mplane;
    model.grain = w.mgrain;
    model.block = w.mblock;
    model.s1 = w.s1;
    model.s2 = w.s2;
    model.vn = w.vn;
    model.v1 = w.v1;
    model.v2 = w.v2;
    model.lam = w.lam;
    model.flags = w.flags;
    model.block_off = job.moff.data();
    int64_t n_model = 0;
    if ((rc = laue_forward_enumerate(geom, planes, &protos, 1, &model, &n_model, w.scratch, w.scratch_bytes, stream)))
        return rc;
    model.n = n_model;
    st.n_model_spots = n_model;
    laue_em_params em = par->em;
    // the likelihood of the final plan at the scoring noise unless given
    if (!(em.sigma_mm > 0.0)) em.sigma_mm = par->score.sigma_mm;
    if (em.eps_cool > 0.0 && !(em.eps_start > 0.0)) {
        // the paper's first temperature (Sec. 7): the farthest of rho = 32 (or
        // em.ot.rho) neighbours keeps a non-negligible weight (laue_eps_init)
        laue_model_spots mk = model;
        mk.n = n_model;
        laue_ot_params on = em.ot;
        on.rho = em.ot.rho > 0 ? em.ot.rho : 32;
        double e0 = 0.0;
        if ((rc = laue_eps_init(geom, obs, &mk, &on, &e0, w.scratch, w.scratch_bytes, stream))) return rc;
        em.eps_start = std::max(e0, em.eps_end);
        log_line("index: eps_init %.4g mm^2", e0);
    }
    const double tb = std::ceil(par->t_b_frac * static_cast<double>(n_model));
    em.ot.t_b = std::max(tb, static_cast<double>(n_model - obs->n));
    const int64_t nf = std::max<int64_t>(obs->n, 1), ng = std::max<int64_t>(n_model, 1);
    k_zero_f<<<static_cast<unsigned>((nf + 255) / 256), 256, 0, s>>>(w.f, nf);
    k_zero_f<<<static_cast<unsigned>((ng + 255) / 256), 256, 0, s>>>(w.g, ng);
    LAUE_CHECK_HIP(hipGetLastError());
    job.protos = protos;
    job.model = model;
    job.em = em;
    job.pot = laue_potentials{w.f, w.g, 0.0, 0.0};
    // the model spots live in the workspace: no per-model-spot output
    job.asg = out->assign;
    job.asg.q_unm = nullptr;
    st.ms_em = ms_since(t0);
    return LAUE_OK;
}

// Whether laue_em_batched takes these EM jobs in one batch: the samples share
// what a batch shares (schedule shape, Gauss-Newton steps, launch, tile,
// chunk, rho and assignment kind) and none asks for the plan-change stop.
bool batchable(const std::vector<EmJob *> &jobs) {
    const laue_em_params &a = jobs[0]->em;
    for (const EmJob *j : jobs) {
        const laue_em_params &b = j->em;
        if (b.eps_cool > 0.0 && b.zeta_tol > 0.0) return false;
        if (b.n_stages != a.n_stages || b.iters_per_stage != a.iters_per_stage || b.gn.k_gn != a.gn.k_gn ||
            b.launch != a.launch || b.tile != a.tile || b.ot.chunk != a.ot.chunk || b.eps_cool != a.eps_cool ||
            b.final_iters != a.final_iters || b.ot.rho != a.ot.rho)
            return false;
        if (em_n_temperatures(b) != em_n_temperatures(a)) return false;
    }
    return true;
}

size_t em_batch_workspace(const std::vector<laue_geometry> &g, const std::vector<int64_t> &no,
                          const std::vector<int64_t> &nm, const std::vector<int32_t> &ng, int32_t rho) {
    const int32_t n = static_cast<int32_t>(g.size());
    return rho > 0 ? laue_sparse_workspace_size(n, g.data(), no.data(), nm.data(), ng.data(), rho)
                   : laue_em_batched_workspace_size(n, g.data(), no.data(), nm.data(), ng.data());
}

// The per-sample storage of laue_index_batched that outlives the front:
// model spots and potentials.
size_t carve_persist(Carver &cv, IndexWs &w, int64_t n_obs, const laue_index_params *p) {
    const int64_t J = std::max<int64_t>(p->max_model_spots, 1);
    w.mplane = cv.take<int>(J);
    w.mgrain = cv.take<int>(J);
    w.mblock = cv.take<int>(J);
    w.s1 = cv.take<float>(J);
    w.s2 = cv.take<float>(J);
    w.vn = cv.take<float>(J);
    w.v1 = cv.take<float>(J);
    w.v2 = cv.take<float>(J);
    w.lam = cv.take<float>(J);
    w.flags = cv.take<uint8_t>(J);
    w.f = cv.take<float>(std::max<int64_t>(n_obs, 1));
    w.g = cv.take<float>(J);
    return cv.size();
}

int validate_index_call(const laue_geometry *geom, const laue_planes *planes, const laue_obs_spots *obs,
                        const laue_index_params *par, const laue_index_out *out) {
    int rc;
    if ((rc = validate_geometry(geom)) || (rc = validate_planes(planes)) || (rc = validate_index_params(par)))
        return rc;
    LAUE_REQUIRE(obs && obs->block_off && obs->n >= 0, LAUE_EINVAL, "detected spots are NULL");
    LAUE_REQUIRE(out && out->q && out->x && out->capacity >= par->k_max, LAUE_EINVAL,
                 "output grains need capacity >= k_max");
    const laue_assignments &as = out->assign;
    const bool with_assign = as.j_star && as.grain && as.q_star && as.q_out;
    LAUE_REQUIRE(with_assign || (!as.j_star && !as.grain && !as.q_star && !as.q_out), LAUE_EINVAL,
                 "assignment arrays must be all given or all NULL");
    return LAUE_OK;
}

}  // namespace
}  // namespace laue

extern "C" int laue_index(const laue_geometry *geom, const laue_planes *planes, const laue_obs_spots *obs,
                          const laue_index_params *par, laue_index_out *out, laue_index_stats *stats, void *ws,
                          size_t ws_bytes, void *stream) {
    clear_error();
    int rc;
    if ((rc = validate_index_call(geom, planes, obs, par, out))) return rc;
    hipStream_t s = static_cast<hipStream_t>(stream);
    Carver cv(ws);
    IndexWs w;
    const size_t need = carve_index(cv, w, geom, planes->n, obs->n, par);
    if ((rc = check_ws(ws, ws_bytes, need))) return rc;
    laue_index_stats st{};
    const auto t_all = std::chrono::steady_clock::now();
    EmJob job{};
    if ((rc = index_front(geom, planes, obs, par, out, w, st, job, s))) return rc;
    if (job.protos.n > 0) {
        const auto t0 = std::chrono::steady_clock::now();
        laue_em_stats es{};
        rc = laue_em(geom, planes, obs, &job.model, &job.em, &job.protos, &job.pot,
                     job.with_assign ? &job.asg : nullptr, &es, w.scratch, w.scratch_bytes, stream);
        if (rc < 0) return rc;
        st.em = es;
        st.ms_em += ms_since(t0);
        log_line("index: EM on %lld model spots, %d iterations, in %.1f ms", static_cast<long long>(job.model.n),
                 es.n_em_iter, st.ms_em);
    }
    st.ms_total = ms_since(t_all);
    if (stats) *stats = st;
    return rc;
}

namespace laue {
namespace {

// Workspace of laue_index_batched: one shared region (each sample's stages
// 1-5a in turn, then the EM of all samples), then every sample's model spots
// and potentials.  Returns the size; with a base, fills shared and persist.
size_t carve_batched(Carver &cv, int32_t n, const laue_geometry *geoms, const int32_t *n_planes,
                     const int64_t *n_obs, const laue_index_params *pars, char **shared, size_t *shared_bytes,
                     std::vector<IndexWs> *persist) {
    size_t front = 0;
    std::vector<laue_geometry> g(geoms, geoms + n);
    std::vector<int64_t> no(n_obs, n_obs + n), nm(n);
    std::vector<int32_t> ng(n);
    for (int k = 0; k < n; ++k) {
        const size_t one = laue_index_workspace_size(geoms + k, n_planes[k], n_obs[k], pars + k);
        if (one == 0) return 0;
        front = std::max(front, one);
        nm[k] = pars[k].max_model_spots;
        ng[k] = pars[k].k_max;
    }
    const size_t em = em_batch_workspace(g, no, nm, ng, pars[0].em.ot.rho);
    if (em == 0) return 0;
    const size_t sh = std::max(front, em);
    char *p = cv.take<char>(sh);
    if (shared) *shared = p;
    if (shared_bytes) *shared_bytes = sh;
    if (persist) persist->assign(n, IndexWs{});
    for (int k = 0; k < n; ++k) {
        IndexWs w{};
        carve_persist(cv, w, n_obs[k], pars + k);
        if (persist) (*persist)[k] = w;
    }
    return cv.size();
}

}  // namespace
}  // namespace laue

extern "C" size_t laue_index_batched_workspace_size(int32_t n, const laue_geometry *geoms, const int32_t *n_planes,
                                                    const int64_t *n_obs, const laue_index_params *pars) {
    if (n < 1 || !geoms || !n_planes || !n_obs || !pars) return 0;
    Carver cv(nullptr);
    return carve_batched(cv, n, geoms, n_planes, n_obs, pars, nullptr, nullptr, nullptr);
}

extern "C" int laue_index_batched(int32_t n, const laue_geometry *geoms, const laue_planes *planes,
                                  const laue_obs_spots *obs, const laue_index_params *pars, laue_index_out *outs,
                                  laue_index_stats *stats, void *ws, size_t ws_bytes, void *stream) {
    clear_error();
    int rc;
    LAUE_REQUIRE(n >= 1 && geoms && planes && obs && pars && outs, LAUE_EINVAL, "NULL argument");
    std::vector<int32_t> npl(n);
    std::vector<int64_t> nob(n);
    for (int k = 0; k < n; ++k) {
        if ((rc = validate_index_call(geoms + k, planes + k, obs + k, pars + k, outs + k))) return rc;
        LAUE_REQUIRE(pars[k].em.ot.rho == pars[0].em.ot.rho, LAUE_EINVAL, "samples of a batch share em.ot.rho");
        npl[k] = planes[k].n;
        nob[k] = obs[k].n;
    }
    const size_t need = laue_index_batched_workspace_size(n, geoms, npl.data(), nob.data(), pars);
    LAUE_REQUIRE(need > 0, LAUE_EINVAL, "invalid index parameters");
    if ((rc = check_ws(ws, ws_bytes, need))) return rc;
    hipStream_t s = static_cast<hipStream_t>(stream);
    Carver cv(ws);
    char *shared = nullptr;
    size_t shared_bytes = 0;
    std::vector<IndexWs> keep;
    carve_batched(cv, n, geoms, npl.data(), nob.data(), pars, &shared, &shared_bytes, &keep);

    // stages 1-5a sample by sample (each fills the GPU on its own), the
    // sample's model spots and potentials in its own storage
    std::vector<laue_index_stats> st(n, laue_index_stats{});
    std::vector<EmJob> jobs(n);
    std::vector<std::chrono::steady_clock::time_point> t_start(n);
    double ms_fronts = 0.0;
    for (int k = 0; k < n; ++k) {
        t_start[k] = std::chrono::steady_clock::now();
        Carver sc(shared);
        IndexWs w;
        carve_index(sc, w, geoms + k, npl[k], nob[k], pars + k);
        const IndexWs &pk = keep[k];
        w.mplane = pk.mplane;
        w.mgrain = pk.mgrain;
        w.mblock = pk.mblock;
        w.s1 = pk.s1;
        w.s2 = pk.s2;
        w.vn = pk.vn;
        w.v1 = pk.v1;
        w.v2 = pk.v2;
        w.lam = pk.lam;
        w.flags = pk.flags;
        w.f = pk.f;
        w.g = pk.g;
        if ((rc = index_front(geoms + k, planes + k, obs + k, pars + k, outs + k, w, st[k], jobs[k], s))) return rc;
        ms_fronts += ms_since(t_start[k]);
    }

    // the EM of every sample with prototypes: one batch when the samples'
    // schedules allow it (laue_em_batched gives each the result of laue_em),
    // else one after another
    std::vector<int> live;
    std::vector<EmJob *> lj;
    for (int k = 0; k < n; ++k)
        if (jobs[k].protos.n > 0) {
            live.push_back(k);
            lj.push_back(&jobs[k]);
        }
    int worst = LAUE_OK;
    const auto t0 = std::chrono::steady_clock::now();
    if (!live.empty() && live.size() > 1 && batchable(lj)) {
        const int m = static_cast<int>(live.size());
        std::vector<laue_geometry> g(m);
        std::vector<laue_planes> pl(m);
        std::vector<laue_obs_spots> ob(m);
        std::vector<laue_model_spots> md(m);
        std::vector<laue_em_params> ep(m);
        std::vector<laue_grains> gr(m);
        std::vector<laue_potentials> pt(m);
        std::vector<laue_assignments> as(m);
        std::vector<laue_em_stats> es(m);
        bool any_assign = false;
        for (int i = 0; i < m; ++i) {
            const int k = live[i];
            g[i] = geoms[k];
            pl[i] = planes[k];
            ob[i] = obs[k];
            md[i] = jobs[k].model;
            ep[i] = jobs[k].em;
            gr[i] = jobs[k].protos;
            pt[i] = jobs[k].pot;
            as[i] = jobs[k].with_assign ? jobs[k].asg : laue_assignments{};
            any_assign = any_assign || jobs[k].with_assign;
        }
        rc = laue_em_batched(m, g.data(), pl.data(), ob.data(), md.data(), ep.data(), gr.data(), pt.data(),
                             any_assign ? as.data() : nullptr, es.data(), shared, shared_bytes, stream);
        if (rc < 0) return rc;
        worst = rc;
        for (int i = 0; i < m; ++i) st[live[i]].em = es[i];
        log_line("index batch: EM of %d samples in one batch, %.1f ms", m, ms_since(t0));
    } else {
        for (int k : live) {
            laue_em_stats es{};
            rc = laue_em(geoms + k, planes + k, obs + k, &jobs[k].model, &jobs[k].em, &jobs[k].protos, &jobs[k].pot,
                         jobs[k].with_assign ? &jobs[k].asg : nullptr, &es, shared, shared_bytes, stream);
            if (rc < 0) return rc;
            worst = std::max(worst, rc);
            st[k].em = es;
        }
        log_line("index batch: EM of %d samples one after another, %.1f ms", static_cast<int>(live.size()),
                 ms_since(t0));
    }
    const double ms_em = ms_since(t0);
    for (int k = 0; k < n; ++k) {
        if (jobs[k].protos.n > 0) st[k].ms_em += ms_em;
        st[k].ms_total = ms_fronts + ms_em;
        if (stats) stats[k] = st[k];
    }
    return worst;
}
