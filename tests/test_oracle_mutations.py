"""The oracle's pins must catch plausible mistakes.

Each case plants one mistake in a copy of the oracle's C source (a flipped sign, a
dropped factor, a transposed or misplaced link, a wrong index), builds it, points the
oracle at the copy and requires that at least one of the named pins fails.  The Python
cases do the same for one function of the oracle's Python face (rebuilt from its
source with the mistake, for that test only).  Nothing here touches the GPU library.
"""
import inspect
import os
import subprocess

import pytest

import oracle as O
import test_oracle_disconnected as TD
import test_oracle_force as TF
import test_oracle_nucleon as TN
import test_oracle_operator as TO
import test_oracle_projection as TP
import test_oracle_solve as TS

MUTATIONS = {
    "projector sign": ("const double sg = (dir > 0) ? -1.0 : 1.0;",
                       "const double sg = (dir > 0) ? 1.0 : -1.0;",
                       [lambda: TO.test_free_field_plane_waves(-1, 0.125)]),
    "antiperiodic sign dropped": ("if (mu == 0 && ((dir > 0 && t == T - 1) || (dir < 0 && t == 0))) ph = (double)bc;",
                                  "if (mu == 0 && ((dir > 0 && t == T - 1) || (dir < 0 && t == 0))) ph = 1.0;",
                                  [lambda: TO.test_free_field_plane_waves(-1, 0.125)]),
    "backward link not daggered": ("W[a][b] = conj(u[3 * b + a]);", "W[a][b] = u[3 * a + b];",
                                   [lambda: TO.test_gauge_covariance(-1)]),
    "backward link at x": ("const long sn = (long)cn[0] * L3 + nsp;", "const long sn = s;",
                           [lambda: TO.test_gauge_covariance(-1)]),
    "mass normalisation": ("const double mass = 1.0 / (2.0 * kappa);", "const double mass = 1.0 / kappa;",
                           [lambda: TO.test_free_field_plane_waves(1, 0.125)]),
    "hop factor": ("res[a][col] -= 0.5 * ph * proj;", "res[a][col] -= ph * proj;",
                   [lambda: TO.test_free_field_plane_waves(1, 0.125)]),
    "gamma_k lower block sign": ("GAMMA[k + 1][2 + a][b] = I * sig[k][a][b];",
                                 "GAMMA[k + 1][2 + a][b] = -I * sig[k][a][b];",
                                 [TO.test_gamma_basis_and_clifford]),
    # a wrong search direction only slows the solver down, because convergence is
    # confirmed on the true residual; a wrong true residual breaks the guarantee
    "true residual": ("cplx d = b[i] - tmp[i];", "cplx d = b[i] - 0.5 * tmp[i];",
                      [lambda: TS.test_solver_vs_lu(-1, None, 0)]),
    "bicgstab residual recursion sign": ("r[i] = s[i] - omega * t[i];", "r[i] = s[i] + omega * t[i];",
                                         [lambda: TS.test_solver_vs_lu(-1, None, 0)]),
    "cgnr without adjoint": ("    ora_gamma5(n / 12, in, tmp);\n    op_apply(A, tmp, out);\n    ora_gamma5(n / 12, out, out);",
                             "    (void)tmp;\n    op_apply(A, in, out);",
                             [lambda: TS.test_solver_vs_lu(-1, None, 1)]),
    "correlator time direction": ("const int ts = mod(t_src + t, T);", "const int ts = mod(t_src - t, T);",
                                  [TS.test_correlator_decays_away_from_source]),
    "force wrap sign dropped": ("gout[3 * r + k] += coeff * ph * g[r][k];", "gout[3 * r + k] += coeff * g[r][k];",
                                [lambda: TF.test_force_vs_finite_differences(-1, (5, 5))]),
    "force outer product transposed": ("g[r][k] += a[s4][r] * conj(Xn[3 * s4 + k]) + Xx[3 * s4 + r] * conj(b[s4][k]);",
                                       "g[r][k] += a[s4][k] * conj(Xn[3 * s4 + r]) + Xx[3 * s4 + r] * conj(b[s4][k]);",
                                       [lambda: TF.test_force_vs_finite_differences(0, None)]),
}


@pytest.mark.slow
@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_planted_mistake_is_caught(name, tmp_path):
    old, new, pins = MUTATIONS[name]
    src = open(O.SRC_PATH).read()
    assert src.count(old) == 1, f"mutation anchor not found once: {name}"
    path = tmp_path / "mutant.c"
    path.write_text(src.replace(old, new))
    so = str(tmp_path / "libmutant.so")
    subprocess.check_call(["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-o", so, str(path), "-lm"])
    prev = O.use_library(so)
    try:
        caught = 0
        for pin in pins:
            try:
                pin()
            except AssertionError:
                caught += 1
        assert caught > 0, f"planted mistake '{name}' passed every pin"
    finally:
        O.restore_library(prev)


# (function, text, replacement, pins)
PY_MUTATIONS = {
    "trace without gamma5": ("disconnected_traces", "gamma5(e), dom=dom", "e, dom=dom",
                             [lambda: TD.test_probing_sources_give_the_exact_trace(-1, None)]),
    "hop term normalisation": ("hop_power", "out = out - 2.0 * kappa * apply_dirac(",
                               "out = out - kappa * apply_dirac(",
                               [lambda: TD.test_probing_sources_give_the_exact_trace(-1, None)]),
    "trace on the wrong slice": ("disconnected_traces", "tau[:, (t0 + k) % T] = prod[:, k]",
                                 "tau[:, (t0 + k + 1) % T] = prod[:, k]",
                                 [lambda: TD.test_probing_sources_give_the_exact_trace(-1, [(3, 2), (1, 2)])]),
    "frontier spin projector sign": ("hop_spin_projector", "(np.eye(4) + sign * g0) / 2", "(np.eye(4) - sign * g0) / 2",
                                     [lambda: TP.test_complete_basis_is_no_approximation(-1)]),
    "projection on the wrong slice": ("_project_slices", "k = (t - t0) % T", "k = (t - t0 + 1) % T",
                                      [TP.test_projected_chain_vs_dense]),
    "charge conjugation gamma_0 only": ("charge_conjugation", "return g[0] @ g[2]", "return g[0]",
                                        [TN.test_block_symmetry_colour_singlet_spin_covariance]),
    "second nucleon contraction with the first one's order": (
        "nucleon_factorized", '"xkija,ab,yijkb->yx"', '"xjika,ab,yijkb->yx"',
        [lambda: TN.test_blocks_equal_the_three_propagator_contraction(5)]),
    "xi not conjugated": ("nucleon_lines", "xi = np.conj(gamma5(z))", "xi = gamma5(z)",
                          [lambda: TN.test_blocks_equal_the_three_propagator_contraction(5)]),
    "frontier term added instead of subtracted": (
        "factorized_propagator", "rhs -= block_apply(U, kappa, T, L, bc, dk, domains[j], hj)",
        "rhs += block_apply(U, kappa, T, L, bc, dk, domains[j], hj)",
        [lambda: TS.test_factorised_chain_vs_dense([(0, 4), (4, 4)], -1)]),
    "chain fed from the source slab only": (
        "factorized_propagator", "if dist[j] == dist[k] - 1:", "if dist[j] == 0:",
        [lambda: TS.test_factorised_chain_vs_dense([(0, 2), (2, 2), (4, 2), (6, 2)], -1)]),
    "overlap grown forward only": ("extended_domain", "return ((t0 - overlap) % T, nt + 2 * overlap)",
                                   "return (t0 % T, nt + overlap)",
                                   [lambda: TS.test_factorised_overlap_vs_dense([(0, 6), (6, 6)], 1, -1)]),
    "two-trace product normalised by n squared": (
        "disconnected_correlator", "return C / (n * (n - 1) * L ** 3)", "return C / (n * n * L ** 3)",
        [lambda: TD.test_two_trace_product_of_noise_free_traces_is_exact(3)]),
    "two-trace product with the i = j terms": (
        "disconnected_correlator", "            if i != j:\n", "            if True:\n",
        [lambda: TD.test_two_trace_product_of_noise_free_traces_is_exact(3),
         TD.test_two_trace_product_is_unbiased_over_every_sign_pattern]),
    "nucleon spin matrix P_- in place of P_+": (
        "nucleon_parity_projector", "return 0.5 * (np.eye(4) + gamma_matrices()[0])",
        "return 0.5 * (np.eye(4) - gamma_matrices()[0])",
        [lambda: TN.test_free_field_nucleon_propagates_forward_with_the_chosen_projector(0.02)]),
    "nucleon spin matrix with the text's gamma5": (
        "nucleon_parity_projector", "return 0.5 * (np.eye(4) + gamma_matrices()[0])",
        "return gamma_matrices()[4] @ (0.5 * (np.eye(4) - gamma_matrices()[0]))",
        [lambda: TN.test_free_field_nucleon_propagates_forward_with_the_chosen_projector(0.02)]),
    "overlap solution crossing from the extension": (
        "factorized_propagator", "hop[k] = xe[:, a:b]", "hop[k] = xe[:, :b - a]",
        [lambda: TS.test_factorised_overlap_vs_dense([(0, 6), (6, 6)], 2, -1)]),
}


@pytest.mark.slow
@pytest.mark.parametrize("name", sorted(PY_MUTATIONS))
def test_planted_python_mistake_is_caught(name, monkeypatch):
    fn, old, new, pins = PY_MUTATIONS[name]
    src = inspect.getsource(getattr(O, fn))
    assert src.count(old) == 1, f"mutation anchor not found once: {name}"
    scope = {}
    exec(compile(src.replace(old, new), f"<mutant {fn}>", "exec"), O.__dict__, scope)
    monkeypatch.setattr(O, fn, scope[fn])
    caught = 0
    for pin in pins:
        try:
            pin()
        except AssertionError:
            caught += 1
    assert caught > 0, f"planted mistake '{name}' passed every pin"
