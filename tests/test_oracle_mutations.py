"""The pins catch plausible mistakes: each case plants one mistake in a copy of
the oracle's C source (on the CPU), builds it, and runs the pin suite against
that build, which must fail."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "lbt1_oracle.c")
SRC3 = os.path.join(ROOT, "oracle", "lbt1_oracle3d.c")

MUTATIONS = {
    "dropped_quadratic_term": ("4.5 * eu * eu", "0.0 * eu * eu"),
    "wrong_sign_u2": ("1.0 - 1.5 * (u * u + v * v)", "1.0 + 1.5 * (u * u + v * v)"),
    "momentum_uses_k_not_inverse": ("us += OR_EX[ik] * f;", "us += OR_EX[k] * f;"),
    "paper_wall_drops_density": ("f = OR_W[ik] * R[x];", "f = OR_W[ik] * 1.0;"),
    "force_not_applied": ("double u = (U[s] + gx) / r;", "double u = U[s] / r;"),
    "halfway_returns_wrong_direction": ("f = oracle_feq(k, r, u, v);", "f = oracle_feq(ik, r, u, v);"),
    "periodic_wrap_transposed": ("ip = (ip + nx) % nx;", "ip = (ip + ny) % ny;"),
    "eu_uses_u_twice": ("double eu = OR_EX[k] * u + OR_EY[k] * v;", "double eu = OR_EX[k] * u + OR_EY[k] * u;"),
    "fixed_nodes_updated": ("if (fl != OR_FLUID) {", "if (fl == OR_SOLID) {"),
    "neighbour_reversed_in_y": ("int jp = j + OR_EY[k];", "int jp = j - OR_EY[k];"),
    "source_density_from_target": ("double r = R[s];", "double r = R[x];"),
    "inverse_table_swapped": ("{0, 3, 4, 1, 2, 7, 8, 5, 6}", "{0, 3, 4, 1, 2, 8, 7, 5, 6}"),
    "diagonal_weight": ("1.0 / 36.0, 1.0 / 36.0};", "1.0 / 36.0, 1.0 / 9.0};"),
    "sc_force_uses_wrong_component": ("sy += OR_W[k] * pk * OR_EY[k];", "sy += OR_W[k] * pk * OR_EX[k];"),
    "sc_force_without_own_psi": ("FX[x] = -G * px * sx;", "FX[x] = -G * sx;"),
    "sc_psi_sign": ("rho0 * (1.0 - exp(-r / rho0))", "rho0 * (1.0 + exp(-r / rho0))"),
    # mistakes in the diagnostics (oracle_reduce)
    "residual_on_momentum_not_velocity": ("double du = fabs(U[x] / R[x] - Us[x] / Rs[x]);",
                                          "double du = fabs(U[x] - Us[x]);"),
    "residual_ignores_y_component": ("if (dv > res) res = dv;", "(void)dv;"),
    "reduce_counts_non_fluid_nodes": ("if (flags && flags[x] != OR_FLUID) continue;",
                                      "if (flags && flags[x] == OR_FIXED) continue;"),
    "mass_of_the_deviation": ("m += R[x];", "m += R[x] - 1.0;"),
    "non_finite_misses_momentum": ("if (!isfinite(R[x]) || !isfinite(U[x]) || !isfinite(V[x])) bad += 1.0;",
                                   "if (!isfinite(R[x])) bad += 1.0;"),
    "residual_against_own_snapshot_density": ("double dv = fabs(V[x] / R[x] - Vs[x] / Rs[x]);",
                                              "double dv = fabs(V[x] / R[x] - Vs[x] / R[x]);"),
}


# mistakes in the 3-D oracle
MUTATIONS3 = {
    "3d_weight_of_edges": ("{1.0 / 3.0, 1.0 / 18.0, 1.0 / 36.0}", "{1.0 / 3.0, 1.0 / 18.0, 1.0 / 18.0}"),
    "3d_momentum_z_from_y": ("ws += L.e[d][2] * f;", "ws += L.e[d][1] * f;"),
    "3d_source_not_upwind": ("long s = nb3(nx, ny, nz, periodic, i, j, k, L.e[id]);",
                             "long s = nb3(nx, ny, nz, periodic, i, j, k, L.e[d]);"),
    "3d_z_wrap": ("c = (c + nz) % nz;", "c = (c + ny) % ny;"),
}


def _build(tmp_path, name, which, old, new):
    srcs = []
    for path in (SRC, SRC3):
        text = open(path).read()
        if path == which:
            assert text.count(old) == 1, name
            text = text.replace(old, new)
        f = tmp_path / os.path.basename(path)
        f.write_text(text)
        srcs.append(str(f))
    lib = tmp_path / "libmutant.so"
    subprocess.run(["gcc", "-O1", "-std=c11", "-fPIC", "-shared", "-ffp-contract=off", "-fopenmp",
                    "-o", str(lib), *srcs, "-lm"], check=True)
    return lib


@pytest.mark.parametrize("name", sorted(MUTATIONS) + sorted(MUTATIONS3))
def test_planted_mistake_fails_a_pin(name, tmp_path):
    which = SRC if name in MUTATIONS else SRC3
    old, new = MUTATIONS.get(name) or MUTATIONS3[name]
    lib = _build(tmp_path, name, which, old, new)
    env = dict(os.environ, LBT1_ORACLE_LIB=str(lib))
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_oracle_pins.py")],
                       env=env, cwd=ROOT, capture_output=True, text=True, timeout=600)
    assert r.returncode != 0, f"mutation {name} survived the pins:\n{r.stdout[-2000:]}"


def test_control_unmodified_copy_passes(tmp_path):
    lib = _build(tmp_path, "control", None, "", "")
    env = dict(os.environ, LBT1_ORACLE_LIB=str(lib))
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_oracle_pins.py")],
                       env=env, cwd=ROOT, capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stdout[-2000:]
