"""Planted mistakes across the oracle: each fails at least one of its pins.

A pin is only as good as the mistakes it catches.  Each case below builds a copy of the oracle
with one plausible mistake (a dropped term, a wrong sign, an off-by-one index, a wrong operand,
a constant of the wrong published method) and runs the pins of that part against it, through
the same checks the pin modules run on the real oracle: the samplers' exact laws (Poisson,
binomial, gamma, GenerateDeparture of Lemma 1 / Algorithm 3) and the log-ratios their rejection
steps accept against (checked against lgamma), Philox against PyTorch's
independent implementation, the scheme order of Section 2.3's tandem example and flow
conservation, closed forms of the M/M/infinity tandem and the exact law of a finite-server
station, and the likelihood-ratio score identities and the exact-chain gradient.  The routing
split and the reach sets have planted mistakes of their own in test_oracle_routing.py and
test_oracle_gradient.py.  test_the_checks_pass_on_the_oracle runs every check on the oracle
itself, so that a failure below is the mistake's and not the check's.
"""
import os
import subprocess

import numpy as np
import pytest
import torch

import oracle
import test_oracle_gradient as tg
import test_oracle_rng_math as trm
import test_oracle_samplers as ts
import test_oracle_schemes as tsc


@pytest.fixture(scope="module")
def aten_exe(tmp_path_factory):
    d = tmp_path_factory.mktemp("aten")
    src, exe = os.path.join(d, "px.cpp"), os.path.join(d, "px")
    open(src, "w").write(trm.ATEN_SRC)
    inc = os.path.join(os.path.dirname(torch.__file__), "include")
    subprocess.run(["g++", "-O1", "-std=c++17", "-I" + inc, "-o", exe, src], check=True)
    return exe


def sampler_checks():
    return {
        "poisson_inversion": lambda: ts.test_poisson(3.3),
        "poisson_ptrs": lambda: ts.test_poisson(37.2),
        "binomial_inversion": lambda: [ts.test_binomial(n, p) for n, p in ((40, 0.2), (560, 0.0999), (150, 0.627),
                                                                        (158, 0.5), (400, 0.19))],
        "binomial_btrs": lambda: [ts.test_binomial(n, p) for n, p in ((1000, 0.2), (800, 0.1), (5000, 0.75))],
        "gamma": lambda: [ts.test_gamma(k) for k in (5, 30)],
        "gendep": lambda: [ts.test_generate_departure_exact_law(*c) for c in
                           ((5, 10, 1.0, 0.5), (12, 12, 1.0, 0.1), (13, 12, 1.5, 0.2), (30, 10, 1.0, 0.05),
                            (30, 10, 2.0, 0.6), (200, 150, 0.5, 0.02))],
        "btrs_log_ratio": lambda: [ts.test_btrs_log_ratio_against_lgamma(n, p) for n, p in ((115, 0.49), (1000, 0.2))],
        "ptrs_log_pmf": lambda: [ts.test_ptrs_log_pmf_against_lgamma(lam) for lam in (10.0, 250.0)],
    }


def scheme_checks():
    return {
        "tandem_trace": tsc.test_paper_tandem_trace,
        "flow_conservation": lambda: [tsc.test_flow_conservation_unit_routing(s) for s in (0, 1)],
        "mminf_closed_form": lambda: [tsc.test_mminf_tandem_closed_form(s, shape) for s in (0, 1) for shape in (0, 1)],
        "finite_server_law": lambda: [tsc.test_finite_server_exact_law(s, 6.0, 1.0, 5, 0.3, 25) for s in (0, 1)],
    }


def score_checks():
    return {
        "departure_scores": lambda: [tg.test_departure_score_identity(*c) for c in
                                     ((4, 6, 1.5, 0.2), (5, 3, 2.0, 0.5), (9, 3, 2.0, 0.3))],
        "arrival_scores": lambda: [tg.test_arrival_score_identity(*c) for c in ((3.7, 0.4), (55.0, 0.25))],
        "exact_chain_gradient": lambda: tg.test_gradient_matches_exact_chain(0, False),
    }


def philox_checks(exe):
    return {"philox_vs_aten": lambda: trm.test_philox_matches_independent_implementation(exe)}


BTRS_TAIL = "- orc_stirling_fc(k) - orc_stirling_fc(n - k);"
KAP_TABLE = "if (kap) kap[i] = (float)(dtd * exp(-(mud * dtd)) / -expm1(-(mud * dtd)));"
BACKWARD_DEP = "for (int32_t i = 0; i < n; ++i) D[i] = departures(c, i, N[i], tau, rep, &ovf, smu);"
BACKWARD_ROUTE = "for (int32_t i = 0; i < n; ++i) route(c, i, D[i], tau, rep, Ain, &ovf, Rrow);"

# name -> (substitutions, family of checks)
MUTANTS = {
    # samplers
    "poisson_inversion_index": ([("p = p * (lam * INV[k]);", "p = p * (lam * INV[k + 1]);")], "sampler"),
    "ptrs_log_sign": ([("- 0.5f * loglam - HALF_LOG_2PI", "+ 0.5f * loglam - HALF_LOG_2PI")], "sampler"),
    "binomial_recurrence_sign": ([("f = f * fmaf(g, INV[k], -r);", "f = f * fmaf(g, INV[k], r);")], "sampler"),
    "binomial_start": ([("float x = (float)n * orc_log1pf(-p);", "float x = -(float)n * p;")], "sampler"),
    "binomial_unscaled_uniform": ([("float u = us_u01(S) * f_from_bits((uint32_t)(sc + 127) << 23);",
                                    "float u = us_u01(S);")], "sampler"),
    "btrs_tail_sign": ([(BTRS_TAIL, "- orc_stirling_fc(k) + orc_stirling_fc(n - k);")], "sampler"),
    "btrs_mode_term": ([("(mf + 0.5f) * orc_log1pf(dm / rnm)", "(mf - 0.5f) * orc_log1pf(dm / rnm)")], "sampler"),
    "btrs_switch_flip": ([("return n - k;\n    }", "return k;\n    }")], "sampler"),
    "gamma_shift": ([("float d = (float)k - 0x1.555556p-2f;", "float d = (float)k - 0.5f;")], "sampler"),
    "gamma_squeeze": ([("0.5f * z2 + d * ((1.0f - v) + orc_logf(v))", "0.5f * z2 + d * ((1.0f - v) - orc_logf(v))")],
                      "sampler"),
    "gendep_split_count": ([("D = orc_binomial(k - 1, dt / T, S);", "D = orc_binomial(k, dt / T, S);")], "sampler"),
    "gendep_erlang_rate": ([("float T = orc_gamma_int(k, S) / rate;", "float T = orc_gamma_int(k, S) / mu;")],
                           "sampler"),
    "gendep_completion_time": ([("float p2 = -orc_expm1f(-(mu * s));", "float p2 = -orc_expm1f(-(mu * dt));")],
                               "sampler"),
    "gendep_drops_offset": ([("D = k + Dp;", "D = Dp;")], "sampler"),
    "gendep_branch_boundary": ([("if (x <= m) {\n        int32_t D = orc_binomial(x, pdep, S);",
                                 "if (x < m) {\n        int32_t D = orc_binomial(x, pdep, S);")], "sampler"),
    # random numbers
    "philox_nine_rounds": ([("for (int round = 0; round < 10; ++round) {", "for (int round = 0; round < 9; ++round) {")],
                           "philox"),
    "philox_key_increment": ([("k1 += PHILOX_W1;", "k1 += PHILOX_W0;")], "philox"),
    "philox_swapped_words": ([("uint32_t y0 = hi1 ^ x1 ^ k0;", "uint32_t y0 = hi0 ^ x1 ^ k0;")], "philox"),
    # schemes
    "backward_same_step_pushes": ([(BACKWARD_DEP + "\n            " + BACKWARD_ROUTE,
                                    "for (int32_t i = 0; i < n; ++i) { D[i] = departures(c, i, N[i] + Ain[i], tau, rep, "
                                    "&ovf, smu); route(c, i, D[i], tau, rep, Ain, &ovf, Rrow); }")], "scheme"),
    "forward_drops_arrivals": ([("int32_t x = N[i] + A[i] + Ain[i];", "int32_t x = N[i] + Ain[i];")], "scheme"),
    "forward_late_pushes": ([("int32_t x = N[i] + A[i] + Ain[i];", "int32_t x = N[i] + A[i];")], "scheme"),
    "sinusoid_integral_sign": ([("(cos(w * t0 + net->phase) - cos(w * t1 + net->phase))",
                                 "(cos(w * t1 + net->phase) - cos(w * t0 + net->phase))")], "scheme"),
    "departure_probability": ([("if (pdep) pdep[i] = (float)(-expm1(-(mud * dtd)));",
                                "if (pdep) pdep[i] = (float)(mud * dtd);")], "scheme"),
    # scores
    "arrival_score_sign": ([("return (float)A / l0 - g;", "return (float)A / l0 + g;")], "score"),
    "binomial_score_count": ([("if (score) *score = (float)D * kap - (float)(x - D) * dt;",
                               "if (score) *score = (float)D * kap - (float)x * dt;")], "score"),
    "erlang_score_shape": ([("float sc = (float)k / mu - (float)m * T;", "float sc = (float)x / mu - (float)m * T;")],
                           "score"),
    "completion_score_term": ([("if (Dp > 0) sc = sc + (float)Dp * (s * (1.0f - p2) / p2);",
                                "if (Dp > 0) sc = sc + (float)Dp * (s / p2);")], "score"),
    "kap_table": ([(KAP_TABLE, "if (kap) kap[i] = (float)(exp(-(mud * dtd)) / -expm1(-(mud * dtd)));")], "score"),
}


def checks_for(family, exe):
    return {"sampler": sampler_checks, "scheme": scheme_checks, "score": score_checks,
            "philox": lambda: philox_checks(exe)}[family]()


def failing_checks(checks):
    failed = []
    for label, check in checks.items():
        try:
            check()
        except AssertionError:
            failed.append(label)
    return failed


def test_the_checks_pass_on_the_oracle(aten_exe):
    for family in ("sampler", "scheme", "score", "philox"):
        assert not failing_checks(checks_for(family, aten_exe)), family


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_planted_mistake_fails_a_pin(name, tmp_path, aten_exe):
    subs, family = MUTANTS[name]
    path = oracle.build_variant(subs, str(tmp_path), f"liboracle_{name}.so")
    with oracle.using_library(path):
        failed = failing_checks(checks_for(family, aten_exe))
    assert failed, f"planted mistake {name} passed every {family} pin"
