"""Plant plausible mistakes in a copy of the oracle and check the pins catch them.

Each mutation edits one spot of ``oracle/oracle.c`` (a tableau entry, the
division of activating terms by lambda, an edge endpoint, a sign, the
inverted sampling of inhibitory lambda, ...), compiles the copy on the CPU,
and runs the pins of ``test_oracle_pins`` (and the step-control pins of
``test_oracle_scipy``, the sampler and Tsit5 pins) against it: at least one
must fail.
"""
import contextlib
import os
import subprocess
import tempfile

import pytest

import oracle
from tests import test_oracle_pins as pins
from tests import test_oracle_scipy as scipy_pins
from tests import test_oracle_sampler as sampler
from tests import test_oracle_tsit5 as tsit5

SRC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "oracle")

# (name, text to replace, replacement, pins expected to catch it)
MUTATIONS = [
    ("tableau a65", "-5103.0 / 18656", "-5103.0 / 18655",
     [pins.test_dp5_fifth_order_on_nonlinear_motif]),
    ("stage input drops h", "s->y[i] = x[i] + h * acc;", "s->y[i] = x[i] + acc;",
     [pins.test_dp5_fifth_order_on_linear_decay, pins.test_dp5_fifth_order_on_nonlinear_motif]),
    ("embedded weight b7", "1.0 / 40};", "1.0 / 41};",
     [pins.test_embedded_error_estimate_scales_as_h5]),
    ("activation not over lambda", "hs = hs / lam;", "hs = hs;",
     [pins.test_hill_at_threshold_is_midpoint, pins.test_hill_limits_and_clamp]),
    ("edge endpoint swapped", "int j = pb->src[e];", "int j = pb->dst[e];",
     [pins.test_hill_limits_and_clamp, pins.test_cascade_fixed_point]),
    ("degradation sign", "- (double)pb->k[i * P + p] * x[i]", "+ (double)pb->k[i * P + p] * x[i]",
     [pins.test_edge_direction_and_degradation]),
    ("hill numerator", "lam * b / (a + b)", "lam * a / (a + b)",
     [pins.test_hill_limits_and_clamp]),
    ("no clamp of negative regulator", "double B = x[j] > 0.0 ? x[j] : 0.0;", "double B = x[j];",
     [pins.test_hill_limits_and_clamp]),
    ("inhibitory lambda not inverted", "l = 1.0 / (inv_lo + (inv_hi - inv_lo) * u);",
     "l = r->lam_inh_min + (r->lam_inh_max - r->lam_inh_min) * u;",
     [pins.test_sampler_distributions]),
    ("median of G/k", "(r->g_min + r->g_max) / (r->k_min + r->k_max)",
     "(r->g_min + r->g_max) / 2.0 / (r->k_min + r->k_max)",
     [pins.test_gk_median_closed_form_and_monte_carlo]),
    ("initial state not scaled by G/k",
     "u * (double)pb->G[i * P + p] / (double)pb->k[i * P + p]", "u * (double)pb->G[i * P + p]",
     [pins.test_unregulated_time_series_matches_closed_form]),
    ("philox mixing", "uint64_t n0 = hi1 ^ c1 ^ k0;", "uint64_t n0 = hi0 ^ c1 ^ k0;",
     [pins.test_philox_matches_numpy_bit_generator]),
    ("hill exponent", "double b = pow(B, n);", "double b = pow(B, n + 1);",
     [pins.test_hill_half_point_for_known_power]),
    ("tsit5 a53 digit", "7.4955393428898365", "7.4955393428998365",
     [tsit5.test_tableau_order_conditions, tsit5.test_tsit5_fifth_order_on_linear_decay]),
    ("tsit5 error weight e4", "-0.1447110071732629,", "-0.1474110071732629,",
     [tsit5.test_tableau_order_conditions]),
    ("tsit5 row 7 weight b6", "2.324710524099774},", "2.324701524099774},",
     [tsit5.test_tableau_order_conditions]),
    ("sobol recurrence drops a term", "uint64_t v = m[k - s] ^ (m[k - s] << s);",
     "uint64_t v = m[k - s] << s;",
     [lambda: sampler.test_sobol_each_dimension_is_a_0m1_net(5),
      lambda: sampler.test_sobol_pairs_meet_the_t_value_bound(3, 7)]),
    ("primitive test skips a factor", "if (orc_gf2_xpow(order / f, poly, s) == 1) return 0;", "",
     [lambda: sampler.test_primitive_polynomial_counts(6)]),
    ("sobol digital shift ignored",
     "return (double)(v ^ orc_sobol_shift(seed, domain, (int32_t)q)) * 0x1.0p-32;",
     "return (double)v * 0x1.0p-32;",
     [sampler.test_sobol_sampler_is_stratified_and_shifted_by_seed]),
    ("lhs jitter dropped", "return ((double)cell + jitter) / (double)lhs_n;",
     "return ((double)cell) / (double)lhs_n;", [sampler.test_lhs_sampler_one_point_per_stratum]),
    ("controller safety factor", "double fac = err > 0 ? 0.9 * pow(err, -1.0 / 5.0) : 10.0;",
     "double fac = err > 0 ? 0.8 * pow(err, -1.0 / 5.0) : 10.0;",
     [lambda: scipy_pins.test_oracle_steps_like_scipy_rk45("er3", 1e-5)]),
    ("controller exponent", "double fac = err > 0 ? 0.9 * pow(err, -1.0 / 5.0) : 10.0;",
     "double fac = err > 0 ? 0.9 * pow(err, -1.0 / 4.0) : 10.0;",
     [lambda: scipy_pins.test_oracle_steps_like_scipy_rk45("er3", 1e-5)]),
    ("rejection factor", "double fac = isfinite(err) ? 0.9 * pow(err, -1.0 / 5.0) : 0.2;",
     "double fac = isfinite(err) ? 0.5 * pow(err, -1.0 / 5.0) : 0.2;",
     [lambda: scipy_pins.test_oracle_steps_like_scipy_rk45("toggle", 0.0)]),
    ("growth not limited after a rejection", "double facmax = last_rejected ? 1.0 : 10.0;",
     "double facmax = 10.0;", [lambda: scipy_pins.test_oracle_steps_like_scipy_rk45("toggle", 0.0)]),
    ("growth limit 5", "double facmax = last_rejected ? 1.0 : 10.0;",
     "double facmax = last_rejected ? 1.0 : 5.0;",
     [lambda: scipy_pins.test_oracle_steps_like_scipy_rk45("er3", 1e-5)]),
    ("starting-step threshold", "(d0 < 1e-5 || d1 < 1e-5)", "(d0 < 1e-10 || d1 < 1e-10)",
     [scipy_pins.test_oracle_starting_step_with_tiny_state]),
    ("starting-step exponent", "pow(0.01 / der, 1.0 / 5.0)", "pow(0.01 / der, 1.0 / 4.0)",
     [lambda: scipy_pins.test_oracle_steps_like_scipy_rk45("cascade", 0.0)]),
    ("steady test drops k_i", "s->o->ss_rtol * (double)s->pb->k[i * P + s->p] * fabs(x[i])",
     "s->o->ss_rtol * fabs(x[i])", [lambda: scipy_pins.test_scaled_steady_stop_closed_form((0.2,))]),
    ("steady test drops the relative term", "s->o->ss_rtol * (double)s->pb->k[i * P + s->p] * fabs(x[i])",
     "0.0 * fabs(x[i])", [lambda: scipy_pins.test_scaled_steady_stop_closed_form((0.15, 0.6, 0.35))]),
    ("real Hill coefficient ignored",
     "double n = pb->nf ? (double)pb->nf[e * P + p] : (double)pb->n[e * P + p];",
     "double n = (double)pb->n[e * P + p];", [pins.test_real_hill_half_point]),
    ("real Hill coefficient range",
     "nf[e * n_sets + j] = (float)((double)r->n_min + (double)(r->n_max - r->n_min) * u);",
     "nf[e * n_sets + j] = (float)((double)r->n_min + (double)(r->n_max) * u);",
     [pins.test_real_hill_sampler_uses_the_integer_draw]),
    ("half-functional activation not over lambda", "if (e < n_act && r->hf_act_over_lambda) h = h / lam;",
     "", [lambda: sampler.test_half_functional_median_matches_independent_monte_carlo(1, 0)]),
]


@contextlib.contextmanager
def mutated_oracle(old, new, tmpdir):
    with open(os.path.join(SRC, "oracle.c")) as f:
        src = f.read()
    assert src.count(old) == 1, f"mutation anchor not unique: {old!r}"
    path_c = os.path.join(tmpdir, "oracle.c")
    with open(path_c, "w") as f:
        f.write(src.replace(old, new))
    with open(os.path.join(SRC, "oracle.h")) as f, open(os.path.join(tmpdir, "oracle.h"), "w") as g:
        g.write(f.read())
    so = os.path.join(tmpdir, "libmut.so")
    subprocess.run(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-ffp-contract=off", "-pthread",
                    path_c, "-o", so, "-lm"], check=True)
    saved = oracle._lib
    oracle._lib = oracle.load(so)
    try:
        yield
    finally:
        oracle._lib = saved


def _fails(fn):
    import inspect
    params = inspect.signature(fn).parameters
    try:
        if "sign" in params and "n" in params:
            fn(sign=-1, n=3)
        elif "sign" in params:
            for s in (1, -1):
                fn(sign=s)
        elif "n" in params:
            fn(n=2)
        elif "builder" in params:
            fn(builder=pins.inputs.toggle_switch)
        elif "method" in params:
            fn(method=oracle.TSIT5)
        else:
            fn()
    except AssertionError:
        return True
    except (ValueError, ZeroDivisionError, FloatingPointError):
        return True
    return False


@pytest.mark.parametrize("name,old,new,catchers", MUTATIONS, ids=[m[0] for m in MUTATIONS])
def test_pins_catch_planted_mistake(name, old, new, catchers):
    with tempfile.TemporaryDirectory() as d, mutated_oracle(old, new, d):
        assert any(_fails(fn) for fn in catchers), f"no pin caught mutation: {name}"


def test_unmutated_copy_passes_the_same_pins():
    # The harness itself must not produce failures.
    with tempfile.TemporaryDirectory() as d, mutated_oracle("int j = pb->src[e];",
                                                            "int j = pb->src[e];", d):
        for _, _, _, catchers in MUTATIONS:
            for fn in catchers:
                assert not _fails(fn), fn.__name__
