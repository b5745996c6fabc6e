"""Planted mistakes: each plausible error in the oracle (a dropped term, a
wrong sign, index or bound, a transposed operand) must make at least one of
the oracle pins in test_oracle.py fail.  Each altered copy of oracle.c is
compiled into a temporary library and the pins run against it in a child
process; nothing here touches the real oracle or any GPU code."""
import os
import subprocess
import sys

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SRC = os.path.join(ROOT, "oracle", "oracle.c")

# (name, original text, planted text, pins that must catch it)
MUTATIONS = [
    ("flip window upper bound", "if (n - dH >= 0 && n - dH <= 12) {", "if (n - dH >= 0 && n - dH < 12) {",
     "local_move or conservation"),
    ("sign of dH", "int dH = 2 * spin(sig[i]) * local_field(g, Js, sig, i);",
     "int dH = -2 * spin(sig[i]) * local_field(g, Js, sig, i);", "local_move or conservation"),
    ("dropped backward bond", "        h += coupling(J[bwd[mu]], mu) * spin(sig[bwd[mu]]);\n", "",
     "local_move or conservation or gauge"),
    ("wrong neighbour index", "int64_t fwd[3] = {site(g, x + 1, y, z), site(g, x, y + 1, z), site(g, x, y, z + 1)};",
     "int64_t fwd[3] = {site(g, x + 1, y, z), site(g, x, y - 1, z), site(g, x, y, z + 1)};",
     "local_move or conservation"),
    ("daemon update sign", "dm[i] = (uint8_t)((n - dH) / 4);", "dm[i] = (uint8_t)((n + dH) / 4);",
     "local_move or conservation"),
    ("energy transposed operand", "H -= coupling(Js[i], mu) * spin(sig[i]) * spin(sig[fwd[mu]]);",
     "H -= coupling(Js[fwd[mu]], mu) * spin(sig[i]) * spin(sig[fwd[mu]]);", "energy or local_move"),
    ("daemon CDF exponent", "expm1(-4.0 * beta * (double)(k + 1))", "expm1(-4.0 * beta * (double)(k))",
     "daemon_thresholds"),
    ("daemon CDF normaliser", "expm1(-16.0 * beta)", "expm1(-12.0 * beta)", "daemon_thresholds"),
    ("heat-bath sign", "exp(-2.0 * beta * h)", "exp(2.0 * beta * h)", "heatbath"),
    ("parity", "return (x + y + z) & 1;", "return (x + y) & 1;", "local_move or order or involution"),
    ("Philox Weyl constant", "#define PHILOX_W1 0xBB67AE85u", "#define PHILOX_W1 0xBB67AE86u", "philox"),
    ("Philox word order", "uint32_t n0 = hi1 ^ c1 ^ k0;", "uint32_t n0 = hi0 ^ c1 ^ k0;", "philox"),
    ("overlap product", "q += spin(sa[i]) * spin(sb[i]);", "q += spin(sa[i]) * spin(sa[i]);", "overlap"),
    ("linear schedule end", "return T0 * (1.0 - f) + T1 * f;", "return T0 * (1.0 - f) + T1;", "schedule"),
    ("log refresh points", "return ((k + 1) & k) == 0;", "return (k & (k - 1)) == 0;", "schedule"),
    ("walker cycle parity", "walker_dir[f], (int)(t & 1), m);", "walker_dir[f], (int)((t + 1) & 1), m);",
     "walkers or wander"),
    ("daemon family draw index", "int64_t j = (int64_t)a * g.N + i;", "int64_t j = i;", "gamma_refresh"),
    ("daemon family in use", "uint8_t *dm = m + (((int64_t)s * R + r) * gamma + alpha) * g.N;",
     "uint8_t *dm = m + (((int64_t)s * R + r) * gamma) * g.N;", "family_alpha or gamma"),
    ("walker family directions", "{0, 2, 4, 1, 3, 5}", "{0, 2, 4, 1, 5, 3}", "wander_along"),
    ("refresh on every sweep of a timestep", "if (a == 0 && oracle_is_refresh(t, P))", "if (oracle_is_refresh(t, P))",
     "gamma_conservation"),
    ("Metropolis tally sign", "sig[i] ^= 1;\n                    acc += dH;", "sig[i] ^= 1;\n                    acc -= dH;",
     "metropolis"),
    ("Metropolis exponent", "floor(exp(-beta * (double)dH) * 4294967296.0)",
     "floor(exp(-0.5 * beta * (double)dH) * 4294967296.0)", "metropolis"),
    ("Metropolis threshold index", "if (u < th[(dH + 12) / 4]) {", "if (u < th[(12 - dH) / 4]) {",
     "metropolis"),
    ("C4 axis of the shift", "site(&g, x + (mu == 0) * r, y + (mu == 1) * r, z + (mu == 2) * r)",
     "site(&g, x + (mu == 1) * r, y + (mu == 0) * r, z + (mu == 2) * r)", "c4"),
    ("C4 replica pairs", "for (int b = a + 1; b < R; b++) {", "for (int b = a; b < R; b++) {", "c4"),
    ("xi ratio", "*xi12 = I[2] / I[1];", "*xi12 = I[2] / I[0];", "xi"),
    ("mesh exponential digit scale", "ldexp(1.0, 8 * d - 17)", "ldexp(1.0, 8 * d - 16)", "pt_exp_digits"),
    ("mesh exponential top digit", ": -expm1(a * (double)(v + 1));", ": -expm1(a * (double)(v));",
     "pt_exp_digits"),
    ("mesh exponential digit word", "c += (uint64_t)w[d] >= t[d * 255 + v];", "c += (uint64_t)w[0] >= t[d * 255 + v];",
     "pt_exp_draw"),
    ("uncapped Creutz bound", "if (n[i] - dH >= 0) {", "if (n[i] - dH > 0) {", "pt_creutz_rule"),
    ("walker update sign", "n[i] -= dH;", "n[i] += dH;", "pt_creutz"),
    ("Gaussian backward bond", "h += (int64_t)Jq[mu * g.N + bwd[mu]] * spin(sig[bwd[mu]]);",
     "h += (int64_t)Jq[mu * g.N + i] * spin(sig[bwd[mu]]);", "pt_delta"),
    ("Houdayer flips one replica", "        sb[queue[q]] ^= 1u;\n", "", "pt_houdayer or pt_equilibrium"),
    ("Houdayer neighbour", "int64_t nb[6] = {site(&g, x + 1, y, z), site(&g, x - 1, y, z),",
     "int64_t nb[6] = {site(&g, x + 1, y, z), site(&g, x + 1, y, z),", "pt_houdayer"),
    ("Houdayer root order", "int64_t k = (int64_t)(((uint64_t)u * (uint64_t)count) >> 32);",
     "int64_t k = count - 1 - (int64_t)(((uint64_t)u * (uint64_t)count) >> 32);", "pt_houdayer"),
    ("tempering swap sign", "if (oracle_pt_exp_draw(pair_tables + (int64_t)t * PT_TABLE, w) >= -x) {",
     "if (oracle_pt_exp_draw(pair_tables + (int64_t)t * PT_TABLE, w) >= x) {", "pt_swap"),
    ("tempering pair order", "for (int t = ph; t + 1 < M; t += 2) {", "for (int t = 0; t + 1 < M; t += 1) {",
     "pt_swap_phase"),
    ("tempering rate", "oracle_pt_exp_table(1.0 / T[t] - 1.0 / T[t + 1],", "oracle_pt_exp_table(1.0 / T[t],",
     "pt_swap_acceptance or pt_equilibrium"),
    ("Metropolis fresh draw per sweep", "philox_words(seed, (uint32_t)i, (uint32_t)k,",
     "philox_words(seed, (uint32_t)i, 0u,", "pt_metropolis"),
    ("all three bonds from output 0",
     "((o[0] >> 31) | ((o[1] >> 31) << 1) | ((o[2] >> 31) << 2))",
     "((o[0] >> 31) | ((o[0] >> 31) << 1) | ((o[0] >> 31) << 2))", "initial_couplings"),
    ("coupling counter without the sample", "(uint32_t)(STREAM_J << 24) | (uint32_t)s};",
     "(uint32_t)(STREAM_J << 24)};", "initial_couplings"),
    ("coupling counter per site word", "uint32_t ctr[4] = {(uint32_t)i, 0u, 0u, (uint32_t)(STREAM_J",
     "uint32_t ctr[4] = {(uint32_t)(i >> 2), 0u, 0u, (uint32_t)(STREAM_J", "initial_couplings"),
    ("spin from output 0", "(uint32_t)(STREAM_SPIN << 24) | (uint32_t)s, (int)(i & 3)) >> 31);",
     "(uint32_t)(STREAM_SPIN << 24) | (uint32_t)s, 0) >> 31);", "initial_spins"),
    ("spins without the replica", "draw(seed, (uint32_t)(i >> 2), 0u, (uint32_t)r,\n",
     "draw(seed, (uint32_t)(i >> 2), 0u, 0u,\n", "initial_spins"),
    ("walker step direction", "{{1, 0, 0}, {-1, 0, 0}, {0, 1, 0}", "{{-1, 0, 0}, {1, 0, 0}, {0, 1, 0}", "walkers"),
]


@pytest.mark.parametrize("name,orig,planted,pins", MUTATIONS, ids=[m[0] for m in MUTATIONS])
def test_planted_mistake_is_caught(name, orig, planted, pins, tmp_path):
    src = open(SRC).read()
    assert src.count(orig) == 1, f"mutation target not found or not unique: {orig!r}"
    mutated = src.replace(orig, planted, 1)
    c = tmp_path / "oracle_mut.c"
    c.write_text(mutated)
    lib = tmp_path / "liboracle_mut.so"
    subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
                           "-o", str(lib), str(c), "-lm"])
    env = dict(os.environ, MICSA_ORACLE_LIB=str(lib), OMP_NUM_THREADS="4")
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        os.path.join(HERE, "test_oracle.py"), "-k", pins],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    # caught means a pin assertion failed (not: no test selected, or a crash)
    assert r.returncode == 1 and " failed" in r.stdout, \
        f"planted mistake '{name}' was not caught by the pins:\n{r.stdout[-2000:]}"
