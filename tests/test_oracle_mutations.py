"""Planted mistakes in the oracle, on the CPU.  Each mutation below is applied
to a copy of oracle/ in a temporary folder (the repository's files are never
touched); the copy's C library is built there and the pin tests that should
notice the mistake run against it in a subprocess, where they must fail.  The
unmutated copy passes the same selections.  This shows that the pins
constrain the oracle where a plausible slip would change it."""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

# (name, file under oracle/, text, replacement, pin file, -k selection)
MUTATIONS = [
    ("philox-multiplier", "muca_oracle.c", "0xD2511F53u", "0xD2511F55u", "test_oracle_pins.py", "known_answers"),
    ("philox-key-schedule", "muca_oracle.c", "k[1] += 0xBB67AE85u;", "k[1] += 0xBB67AE86u;",
     "test_oracle_pins.py", "known_answers"),
    ("bond-count", "muca_oracle.c", "if (s[i] != s[nb[2]]) ++k;", "if (s[i] != s[nb[0]]) ++k;",
     "test_oracle_pins.py", "kaufman_beale"),
    ("ising-reachable", "muca_oracle.c", "r = (k % 2 == 0) && k != 2 && k != 2 * N - 2;",
     "r = (k % 2 == 0) && k != 2;", "test_oracle_pins.py", "beale_invariants"),
    ("recursion-sign", "muca_oracle.c", "if (H[b] > 0) lnW[b] -= log((double)H[b]);",
     "if (H[b] > 0) lnW[b] += log((double)H[b]);", "test_oracle_pins.py", "converges_to_exact_dos_ising_L4"),
    ("norm-sum-not-mean", "muca_oracle.c", "const double mean = n > 0 ? sum / n : 0.0;",
     "const double mean = n > 0 ? sum : 0.0;", "test_oracle_pins.py", "normalized"),
    ("norm-mean-over-all-bins", "muca_oracle.c", "const double mean = n > 0 ? sum / n : 0.0;",
     "const double mean = n > 0 ? sum / n_bins : 0.0;", "test_oracle_pins.py", "normalized"),
    ("norm-shift-sign", "muca_oracle.c", "if (H[b] > 0) lnW[b] -= log((double)H[b]) - mean;",
     "if (H[b] > 0) lnW[b] -= log((double)H[b]) + mean;", "test_oracle_pins.py", "normalized"),
    ("correction-slope", "__init__.py", "slope = (lnW[lo] - lnW[a]) / float(lo - a)",
     "slope = (lnW[lo] - lnW[a]) / float(a - lo)", "test_oracle_pins.py", "correction"),
    ("dk-sign", "muca_oracle.c", "int dk = after - before;", "int dk = before - after;",
     "test_oracle_pins.py", "tracked_state"),
    ("table-direction", "muca_oracle.c", "v = threshold_of(lnW[t] - lnW[k]);", "v = threshold_of(lnW[k] - lnW[t]);",
     "test_oracle_pins.py", "table_"),
    ("potts-proposal-range", "muca_oracle.c", "(uint64_t)(j->q - 1)) >> 32);", "(uint64_t)(j->q)) >> 32);",
     "test_oracle_pins.py", "infinite_temperature"),
    ("up-neighbour", "muca_oracle.c", "nb[3] = ((y + L - 1) % L) * L + x; /* up    */",
     "nb[3] = ((y + L - 1) % L) * L + (x + 1) % L; /* up    */", "test_oracle_pins.py", "tracked_state"),
    ("abs-m", "muca_oracle.c",
     "if (j->record == REC_PROD) j->sabs[(size_t)c * j->n_bins + k] += (m < 0) ? -m : m;",
     "if (j->record == REC_PROD) j->sabs[(size_t)c * j->n_bins + k] += m;",
     "test_oracle_reweight.py", "production_run"),
    ("mag-beta-sign", "muca_oracle.c", "- beta * (double)(2 * dk))", "+ beta * (double)(2 * dk))",
     "test_oracle_mag.py", "canonical_magnetization"),
    ("mag-spin-columns", "muca_oracle.c", "(s[i] ? 5 : 0)]", "(s[i] ? 0 : 5)]",
     "test_oracle_mag.py", "canonical_magnetization"),
    ("mag-factor-2", "muca_oracle.c", "- beta * (double)(2 * dk))", "- beta * (double)(dk))",
     "test_oracle_mag.py", "canonical_magnetization"),
    ("mag-k-sum", "muca_oracle.c", "if (j->record == REC_PROD) j->sabs[(size_t)c * j->n_bins + b] += k;",
     "if (j->record == REC_PROD) j->sabs[(size_t)c * j->n_bins + b] += k + 1;",
     "test_oracle_mag.py", "canonical_magnetization"),
    ("mag-dk-column", "muca_oracle.c", "(dk + 4) / 2 + (s[i]", "(4 - dk) / 2 + (s[i]",
     "test_oracle_mag.py", "canonical_magnetization"),
    ("mag-enumeration-energy", "muca_oracle.c", "double w = exp(-beta * ((-2.0 * N + 2.0 * k) - e_ground));",
     "double w = exp(-beta * ((-2.0 * N + 1.0 * k) - e_ground));", "test_oracle_mag.py", "transfer_matrix"),
    ("mag-m-direction", "muca_oracle.c", "int t = u ? m - 1 : m + 1;", "int t = u ? m + 1 : m - 1;",
     "test_oracle_mag.py", "canonical_magnetization or detailed_balance"),
    ("reweight-lnw-sign", "__init__.py", "a = np.log(ck) - lw - beta * Ek", "a = np.log(ck) + lw - beta * Ek",
     "test_oracle_reweight.py", "kaufman or potts"),
    ("potts-energy", "__init__.py", "return -2.0 * N + (2.0 * k if model == ISING else k)", "return -2.0 * N + 2.0 * k",
     "test_oracle_reweight.py", "potts"),
    ("flatness-strict", "__init__.py", "flat = covered and mom >= ratio", "flat = covered and mom > ratio",
     "test_oracle_pins.py", "flatness"),
    ("eqh-beta-sign", "__init__.py", "- beta * E[ks]", "+ beta * E[ks]",
     "test_oracle_interface.py", "closed_form"),
    ("eqh-bisection", "__init__.py", "if gap(mid) < 0.0:", "if gap(mid) > 0.0:",
     "test_oracle_interface.py", "closed_form"),
    ("eqh-one-over-l", "__init__.py", "/ (2.0 * L), ks", "/ (1.0 * L), ks",
     "test_oracle_interface.py", "closed_form"),
    ("eqh-drop-ln-cnt", "__init__.py", "a = np.log(np.asarray(cnt, np.float64)[ks]) - ",
     "a = 0.0 * np.log(np.asarray(cnt, np.float64)[ks]) - ", "test_oracle_interface.py", "uses_the_counts"),
    ("eqh-plain-valley", "__init__.py",
     "score = np.minimum(left, right) - a - np.abs(np.log(m_left) - np.log(m_right))",
     "score = np.minimum(left, right) - a", "test_oracle_interface.py", "sparse_tail"),
    ("eqh-height-balance", "__init__.py",
     "score = np.minimum(left, right) - a - np.abs(np.log(m_left) - np.log(m_right))",
     "score = np.minimum(left, right) - a - np.abs(left - right)", "test_oracle_interface.py",
     "ground_state or sparse_tail"),
    ("eqh-split-moves-with-beta", "__init__.py", "low, high = ks <= split, ks > split",
     "mean = int(np.average(ks, weights=np.exp(a - a.max()))); low, high = ks <= mean, ks > mean",
     "test_oracle_interface.py", "wide_bracket"),
    ("gelu-coefficient", "mlp_ref.py", "t = np.tanh(_C * (z + 0.044715 * z ** 3))", "t = np.tanh(_C * (z + 0.04 * z ** 3))",
     "test_oracle_mlp.py", "gelu"),
    ("gelu-derivative", "mlp_ref.py", "(1.0 + 3 * 0.044715 * z * z)", "(1.0 + 2 * 0.044715 * z * z)",
     "test_oracle_mlp.py", "gelu or finite_differences"),
    ("adam-correction-off-by-one", "mlp_ref.py", "vh = v / (1 - b2 ** step)", "vh = v / (1 - b2 ** (step + 1))",
     "test_oracle_mlp.py", "adam"),
    ("adam-no-correction", "mlp_ref.py", "mh = m / (1 - b1 ** step)", "mh = m", "test_oracle_mlp.py", "adam"),
    ("adam-rates-swapped", "mlp_ref.py", "def adam(p, g, m, v, step, lr, b1=0.9, b2=0.999, eps=1e-8):",
     "def adam(p, g, m, v, step, lr, b1=0.999, b2=0.9, eps=1e-8):", "test_oracle_mlp.py", "adam"),
]


def _copy(tmp, pin_file):
    shutil.copytree(os.path.join(ROOT, "oracle"), os.path.join(tmp, "oracle"),
                    ignore=shutil.ignore_patterns("*.so", "*.tmp", "__pycache__"))
    os.makedirs(os.path.join(tmp, "tests"))
    for f in ("conftest.py", "exact_ising.py", pin_file):
        shutil.copy(os.path.join(ROOT, "tests", f), os.path.join(tmp, "tests", f))
    shutil.copytree(os.path.join(ROOT, "tests", "golden"), os.path.join(tmp, "tests", "golden"))


def _run(tmp, pin_file, selection):
    return subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider", "-k", selection,
                           os.path.join(tmp, "tests", pin_file)], cwd=tmp, capture_output=True, text=True,
                          timeout=600)


@pytest.mark.parametrize("name,fname,old,new,pin_file,selection", MUTATIONS, ids=[m[0] for m in MUTATIONS])
def test_planted_mistake_fails_a_pin(tmp_path, name, fname, old, new, pin_file, selection):
    tmp = str(tmp_path)
    _copy(tmp, pin_file)
    path = os.path.join(tmp, "oracle", fname)
    src = open(path).read()
    assert src.count(old) == 1, f"{name}: the text to mutate must occur exactly once"
    with open(path, "w") as fh:
        fh.write(src.replace(old, new))
    res = _run(tmp, pin_file, selection)
    # exit status 1: tests ran and at least one failed (2-5 would be errors or nothing collected)
    assert res.returncode == 1 and " failed" in res.stdout, res.stdout[-3000:] + res.stderr[-2000:]


@pytest.mark.parametrize("pin_file", sorted({m[4] for m in MUTATIONS}))
def test_unmutated_copy_passes_the_same_selections(tmp_path, pin_file):
    tmp = str(tmp_path)
    _copy(tmp, pin_file)
    selection = " or ".join(sorted({f"({m[5]})" for m in MUTATIONS if m[4] == pin_file}))
    res = _run(tmp, pin_file, selection)
    assert res.returncode == 0 and " passed" in res.stdout, res.stdout[-3000:] + res.stderr[-2000:]
