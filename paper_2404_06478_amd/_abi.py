"""ctypes mirror of include/laueot.h (structs, codes, prototypes)."""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblaueot.so")

LAUE_OK = 0
LAUE_ENOCONV = 1
LAUE_EINVAL = -1
LAUE_EINFEASIBLE = -2
LAUE_ECAPACITY = -3
LAUE_EDEVICE = -4
LAUE_EWORKSPACE = -5
MAX_DET = 4
MAX_ROT = 360

vp = C.c_void_p
d3 = C.c_double * 3


class laue_detector(C.Structure):
    _fields_ = [("center", d3), ("normal", d3), ("axis1", d3), ("axis2", d3), ("half_size", C.c_double)]


class laue_geometry(C.Structure):
    _fields_ = [("n_rot", C.c_int32), ("n_det", C.c_int32), ("omega0", C.c_double),
                ("domega", C.c_double), ("lambda_min", C.c_double), ("lambda_max", C.c_double),
                ("det", laue_detector * MAX_DET)]


class laue_planes(C.Structure):
    _fields_ = [("n", C.c_int32), ("w", vp), ("d", vp), ("harmonic_prev", vp)]


class laue_grains(C.Structure):
    _fields_ = [("n", C.c_int32), ("q", vp), ("x", vp)]


class laue_obs_spots(C.Structure):
    _fields_ = [("n", C.c_int64), ("p1", vp), ("p2", vp), ("block_off", vp)]


class laue_model_spots(C.Structure):
    _fields_ = [("n", C.c_int64), ("plane", vp), ("grain", vp), ("block", vp), ("s1", vp),
                ("s2", vp), ("vn", vp), ("v1", vp), ("v2", vp), ("lam", vp), ("flags", vp),
                ("block_off", vp)]


class laue_ot_params(C.Structure):
    _fields_ = [("eps", C.c_double), ("distance", C.c_double), ("c_out", C.c_double),
                ("c_unm", C.c_double), ("c_sink", C.c_double), ("t_b", C.c_double),
                ("tol", C.c_double), ("n_max", C.c_int32), ("chunk", C.c_int32), ("rho", C.c_int32),
                ("outlier_model", C.c_int32), ("kappa", C.c_double), ("lam", C.c_double),
                ("m_frac", C.c_double)]


class laue_potentials(C.Structure):
    _fields_ = [("f", vp), ("g", vp), ("f0", C.c_double), ("g0", C.c_double)]


class laue_objective(C.Structure):
    _fields_ = [("mass", C.c_double), ("cost_inlier", C.c_double), ("cost_total", C.c_double),
                ("entropy", C.c_double), ("sem_objective", C.c_double)]


class laue_ot_stats(C.Structure):
    _fields_ = [("n_iter", C.c_int32), ("converged", C.c_int32), ("err", C.c_double)]


class laue_gn_params(C.Structure):
    _fields_ = [("k_gn", C.c_int32), ("mu_rel", C.c_double), ("method", C.c_int32), ("k_newton", C.c_int32),
                ("k_mm", C.c_int32), ("tol_x", C.c_double), ("tol_r", C.c_double)]


class laue_em_params(C.Structure):
    _fields_ = [("ot", laue_ot_params), ("gn", laue_gn_params), ("eps_start", C.c_double),
                ("eps_end", C.c_double), ("n_stages", C.c_int32), ("iters_per_stage", C.c_int32),
                ("launch", C.c_int32), ("tile", C.c_int32), ("eps_cool", C.c_double),
                ("final_iters", C.c_int32), ("zeta_tol", C.c_double), ("sigma_mm", C.c_double)]


class laue_em_stats(C.Structure):
    _fields_ = [("n_em_iter", C.c_int32), ("sinkhorn_iters", C.c_int64),
                ("cost_entries", C.c_int64), ("not_converged", C.c_int32), ("last_err", C.c_double),
                ("sinkhorn_ms", C.c_double), ("sinkhorn_passes", C.c_int64),
                ("sinkhorn_entries", C.c_int64), ("mstep_ms", C.c_double),
                ("mstep_entries", C.c_int64), ("launch_used", C.c_int32), ("polls", C.c_int32),
                ("tile2_solves", C.c_int32), ("objective", laue_objective), ("zeta", C.c_double),
                ("final_iters_run", C.c_int32)]


class laue_assignments(C.Structure):
    _fields_ = [("j_star", vp), ("grain", vp), ("q_star", vp), ("q_out", vp), ("q_unm", vp)]


class laue_cand_params(C.Structure):
    _fields_ = [("n_pairs", C.c_int64), ("seed", C.c_uint64), ("delta_deg", C.c_double), ("pair_a", vp),
                ("pair_b", vp)]


class laue_candidates(C.Structure):
    _fields_ = [("n", C.c_int64), ("q", vp), ("pair", vp), ("ma", vp), ("mb", vp), ("spot_a", vp),
                ("spot_b", vp), ("feat", vp)]


class laue_score_params(C.Structure):
    _fields_ = [("sigma_mm", C.c_double), ("distance", C.c_double), ("c_out", C.c_double),
                ("f_out", C.c_double), ("eps_start", C.c_double), ("eps_end", C.c_double),
                ("k_refine", C.c_int32), ("k_gn", C.c_int32), ("mu_rel", C.c_double),
                ("chunk", C.c_int32), ("max_spots_per_cand", C.c_int32), ("eps_cool", C.c_double),
                ("drop_log2", C.c_double)]


class laue_score_out(C.Structure):
    _fields_ = [("n_model", vp), ("n_unmatched", vp), ("keep", vp), ("lbar_off", vp),
                ("lbar_row", vp), ("lbar_val", vp), ("lbar_cap", C.c_int64), ("lbar_n", C.c_int64),
                ("pairs_streamed", C.c_int64), ("pairs_evaluated", C.c_int64),
                ("pairs_refine", C.c_int64)]


class laue_mlp(C.Structure):
    _fields_ = [("n_in", C.c_int32), ("n_hidden", C.c_int32), ("params", vp), ("wbf16", vp),
                ("adam_m", vp), ("adam_v", vp), ("step", C.c_int32)]


class laue_support_params(C.Structure):
    _fields_ = [("radius_mm", C.c_double), ("n_support_planes", C.c_int32)]


class laue_adam_params(C.Structure):
    _fields_ = [("lr", C.c_double), ("beta1", C.c_double), ("beta2", C.c_double), ("eps", C.c_double)]


LAUE_INDEX_PLAIN = 0
LAUE_INDEX_LEARNED = 1
LAUE_INDEX_SOBOL = 2


class laue_sobol_params(C.Structure):
    _fields_ = [("first", C.c_int64), ("mrp_half", C.c_double), ("x_half", C.c_double * 3),
                ("restrict_fz", C.c_int32)]


class laue_index_params(C.Structure):
    _fields_ = [("mode", C.c_int32), ("cand", laue_cand_params), ("max_candidates", C.c_int64),
                ("mlp", C.POINTER(laue_mlp)), ("support", laue_support_params), ("top_frac", C.c_double),
                ("score", laue_score_params), ("lbar_cap", C.c_int64), ("k_max", C.c_int32),
                ("max_model_spots", C.c_int64), ("t_b_frac", C.c_double), ("em", laue_em_params),
                ("sobol", laue_sobol_params)]


class laue_index_stats(C.Structure):
    _fields_ = [("n_candidates_found", C.c_int64), ("n_candidates", C.c_int64), ("n_scored", C.c_int64),
                ("lbar_entries", C.c_int64), ("n_picked", C.c_int32), ("n_prototypes", C.c_int32),
                ("n_model_spots", C.c_int64), ("ms_candidates", C.c_double), ("ms_proposal", C.c_double),
                ("ms_score", C.c_double), ("ms_greedy", C.c_double), ("ms_em", C.c_double),
                ("ms_total", C.c_double), ("em", laue_em_stats), ("score_pairs", C.c_int64),
                ("score_pairs_evaluated", C.c_int64), ("score_pairs_refine", C.c_int64)]


class laue_index_out(C.Structure):
    _fields_ = [("capacity", C.c_int32), ("n_grains", C.c_int32), ("q", vp), ("x", vp),
                ("assign", laue_assignments)]


P = C.POINTER
SIGNATURES = {
    "laue_version": (C.c_int, []),
    "laue_last_error": (C.c_char_p, []),
    "laue_planes_cubic": (C.c_int, [C.c_double, C.c_char, C.c_int, P(C.c_int32), vp, vp, vp, vp]),
    "laue_forward_workspace_size": (C.c_size_t, [P(laue_geometry), C.c_int32, C.c_int32]),
    "laue_forward_enumerate": (C.c_int, [P(laue_geometry), P(laue_planes), P(laue_grains), C.c_int,
                                         P(laue_model_spots), P(C.c_int64), vp, C.c_size_t, vp]),
    "laue_forward_enumerate_counted": (C.c_int, [P(laue_geometry), P(laue_planes), P(laue_grains), C.c_int,
                                                 P(laue_model_spots), P(C.c_int64), vp, C.c_size_t, vp]),
    "laue_forward_eval": (C.c_int, [P(laue_geometry), P(laue_planes), P(laue_grains),
                                    P(laue_model_spots), vp, C.c_size_t, vp]),
    "laue_simulate_workspace_size": (C.c_size_t, [P(laue_geometry), C.c_int32, C.c_int32, C.c_int64,
                                                  C.c_int64]),
    "laue_simulate": (C.c_int, [P(laue_geometry), P(laue_planes), P(laue_grains), C.c_double,
                                C.c_double, C.c_double, C.c_uint64, C.c_int64, vp, vp, vp, vp, vp,
                                P(C.c_int64), vp, C.c_size_t, vp]),
    "laue_sinkhorn_workspace_size": (C.c_size_t, [P(laue_geometry), C.c_int64, C.c_int64, C.c_int32]),
    "laue_sinkhorn": (C.c_int, [P(laue_geometry), P(laue_obs_spots), P(laue_model_spots),
                                P(laue_ot_params), P(laue_potentials), P(laue_ot_stats), vp,
                                C.c_size_t, vp]),
    "laue_plan_block": (C.c_int, [P(laue_geometry), P(laue_obs_spots), P(laue_model_spots),
                                  P(laue_ot_params), P(laue_potentials), C.c_int32, vp, vp]),
    "laue_cost_block": (C.c_int, [P(laue_geometry), P(laue_obs_spots), P(laue_model_spots),
                                  C.c_double, C.c_int32, vp, vp]),
    "laue_mstep": (C.c_int, [P(laue_geometry), P(laue_planes), P(laue_obs_spots),
                             P(laue_model_spots), P(laue_ot_params), P(laue_potentials),
                             P(laue_gn_params), P(laue_grains), vp, vp, C.c_size_t, vp]),
    "laue_em": (C.c_int, [P(laue_geometry), P(laue_planes), P(laue_obs_spots), P(laue_model_spots),
                          P(laue_em_params), P(laue_grains), P(laue_potentials),
                          P(laue_assignments), P(laue_em_stats), vp, C.c_size_t, vp]),
    "laue_candidates_workspace_size": (C.c_size_t, [P(laue_geometry), C.c_int32, C.c_int64]),
    "laue_candidates_generate": (C.c_int, [P(laue_geometry), P(laue_planes), P(laue_obs_spots),
                                           P(laue_cand_params), P(laue_candidates), P(C.c_int64), vp,
                                           C.c_size_t, vp]),
    "laue_score_workspace_size": (C.c_size_t, [P(laue_geometry), C.c_int64, P(laue_score_params)]),
    "laue_score_candidates": (C.c_int, [P(laue_geometry), P(laue_planes), P(laue_obs_spots),
                                        P(laue_grains), P(laue_score_params), P(laue_score_out), vp,
                                        C.c_size_t, vp]),
    "laue_spot_greedy_workspace_size": (C.c_size_t, [C.c_int32, C.c_int64]),
    "laue_spot_greedy": (C.c_int, [vp, vp, vp, C.c_int32, C.c_int64, C.c_double, C.c_int32, vp, vp,
                                   P(C.c_int32), vp, C.c_size_t, vp]),
    "laue_mlp_n_params": (C.c_int64, [C.c_int32, C.c_int32]),
    "laue_mlp_n_bf16": (C.c_int64, [C.c_int32, C.c_int32]),
    "laue_mlp_init": (C.c_int, [P(laue_mlp), C.c_uint64, vp]),
    "laue_mlp_sync_bf16": (C.c_int, [P(laue_mlp), vp]),
    "laue_mlp_forward_workspace_size": (C.c_size_t, [C.c_int64]),
    "laue_mlp_forward": (C.c_int, [P(laue_mlp), vp, C.c_int64, vp, vp, C.c_size_t, vp]),
    "laue_mlp_train_workspace_size": (C.c_size_t, [C.c_int64]),
    "laue_mlp_backward": (C.c_int, [P(laue_mlp), vp, vp, C.c_int64, vp, P(C.c_double), vp, C.c_size_t, vp]),
    "laue_mlp_adam": (C.c_int, [P(laue_mlp), vp, P(laue_adam_params), vp]),
    "laue_mlp_train_step": (C.c_int, [P(laue_mlp), vp, vp, C.c_int64, P(laue_adam_params), P(C.c_double), vp,
                                      C.c_size_t, vp]),
    "laue_candidate_support_workspace_size": (C.c_size_t, [P(laue_geometry), C.c_int32, C.c_int64,
                                                           P(laue_support_params)]),
    "laue_candidate_support": (C.c_int, [P(laue_geometry), P(laue_planes), P(laue_obs_spots), P(laue_candidates),
                                         P(laue_support_params), vp, C.c_size_t, vp]),
    "laue_candidate_labels": (C.c_int, [P(laue_candidates), vp, C.c_int64, P(laue_grains), C.c_double, vp, vp,
                                        vp]),
    "laue_candidate_labels_nearest": (C.c_int, [P(laue_candidates), P(laue_grains), C.c_double, vp, vp, vp,
                                                vp]),
    "laue_pairs_same_grain": (C.c_int, [P(laue_geometry), P(laue_obs_spots), vp, C.c_int64, C.c_uint64, vp, vp,
                                        vp, C.c_size_t, vp]),
    "laue_pairs_same_grain_workspace_size": (C.c_size_t, [P(laue_geometry)]),
    "laue_index_workspace_size": (C.c_size_t, [P(laue_geometry), C.c_int32, C.c_int64, P(laue_index_params)]),
    "laue_index": (C.c_int, [P(laue_geometry), P(laue_planes), P(laue_obs_spots), P(laue_index_params),
                             P(laue_index_out), P(laue_index_stats), vp, C.c_size_t, vp]),
    "laue_index_batched_workspace_size": (C.c_size_t, [C.c_int32, P(laue_geometry), vp, vp,
                                                        P(laue_index_params)]),
    "laue_index_batched": (C.c_int, [C.c_int32, P(laue_geometry), P(laue_planes), P(laue_obs_spots),
                                     P(laue_index_params), P(laue_index_out), P(laue_index_stats), vp, C.c_size_t,
                                     vp]),
    "laue_em_batched_workspace_size": (C.c_size_t, [C.c_int32, P(laue_geometry), vp, vp, vp]),
    "laue_sparse_workspace_size": (C.c_size_t, [C.c_int32, P(laue_geometry), vp, vp, vp, C.c_int32]),
    "laue_sobol_workspace_size": (C.c_size_t, [C.c_int64]),
    "laue_objectives": (C.c_int, [P(laue_geometry), P(laue_obs_spots), P(laue_model_spots), P(laue_ot_params),
                                  P(laue_potentials), C.c_double, P(laue_objective), vp, C.c_size_t, vp]),
    "laue_sobol_starts": (C.c_int, [P(laue_sobol_params), C.c_int64, vp, vp, P(C.c_int64), vp, C.c_size_t, vp]),
    "laue_sparse_neighbors": (C.c_int, [P(laue_geometry), P(laue_obs_spots), P(laue_model_spots), P(laue_ot_params),
                                        vp, vp, P(C.c_int64), vp, C.c_size_t, vp]),
    "laue_em_batched": (C.c_int, [C.c_int32, P(laue_geometry), P(laue_planes), P(laue_obs_spots),
                                  P(laue_model_spots), P(laue_em_params), P(laue_grains), P(laue_potentials),
                                  P(laue_assignments), P(laue_em_stats), vp, C.c_size_t, vp]),
    "laue_ot_defaults": (C.c_int, [C.c_double, C.c_double, C.c_int64, P(laue_ot_params)]),
    "laue_mlp_epoch_workspace_size": (C.c_size_t, [C.c_int64, C.c_int64]),
    "laue_mlp_train_epoch": (C.c_int, [P(laue_mlp), vp, vp, C.c_int64, C.c_int64, C.c_uint64, C.c_int32,
                                       P(laue_adam_params), P(C.c_double), vp, C.c_size_t, vp]),
    "laue_sinkhorn_noalloc_capacity": (C.c_size_t, []),
    "laue_sinkhorn_noalloc": (C.c_int, [P(laue_geometry), P(laue_obs_spots), P(laue_model_spots),
                                        P(laue_ot_params), P(laue_potentials), P(laue_ot_stats), vp]),
    "laue_eps_init": (C.c_int, [P(laue_geometry), P(laue_obs_spots), P(laue_model_spots), P(laue_ot_params),
                                P(C.c_double), vp, C.c_size_t, vp]),
    "laue_select_top_workspace_size": (C.c_size_t, [C.c_int64]),
    "laue_select_top": (C.c_int, [vp, C.c_int64, C.c_int64, vp, vp, C.c_size_t, vp]),
}


def load(path: str = LIB_PATH) -> C.CDLL:
    lib = C.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib
