"""The oracle pins catch plausible mistakes: each case below plants one mistake
in a copy of the oracle's C source (never in the oracle itself), builds it,
and runs the pins against that build, which must fail.  CPU only.

The mistakes are of the kinds a reading of Sec. 3 could make: a wrong sign,
a dropped term, a wrong factor, a wrong stencil or comparison, the history
seen from the wrong side.  A control build of the unchanged source passes.
"""
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "dem_oracle.c")

# name: (what it breaks, text in the oracle, the planted replacement)
MUTATIONS = {
    "spin_sign": ("Eq. 4: relative surface velocity uses r_i w_i + r_j w_j",
                  "G->spin[k] = s->r[a] * s->w[3 * a + k] + s->r[b] * s->w[3 * b + k];",
                  "G->spin[k] = s->r[a] * s->w[3 * a + k] - s->r[b] * s->w[3 * b + k];"),
    "no_projection": ("Eq. 7: delta_t projected onto the tangent plane",
                      "dt_new[k] = h[k] - hn * G->n[k] + vt[k] * p->dt;",
                      "dt_new[k] = h[k] + vt[k] * p->dt;"),
    "torque_b_sign": ("Eq. 3: torque on the partner",
                      "T[3 * b + q] += s->r[b] * nxft[q] - Cr[q];",
                      "T[3 * b + q] += -s->r[b] * nxft[q] - Cr[q];"),
    "torque_scale": ("Eq. 3: torque lever arm r_i",
                     "T[3 * a + q] += s->r[a] * nxft[q] + Cr[q];",
                     "T[3 * a + q] += s->r[a] * nxft[q] * 1.0001 + Cr[q];"),
    "eta_mass": ("Eq. 10: eta = alpha sqrt(k M)",
                 "double eta = K->alpha * sqrt(kn * G->M);",
                 "double eta = K->alpha * sqrt(kn * G->M * 2.0);"),
    "alpha_factor": ("Eq. 10: alpha from the restitution coefficient",
                     "-2.0 * log(e) / sqrt",
                     "-1.0 * log(e) / sqrt"),
    "no_cap_rescale": ("Eq. 5: delta_t rescaled when the Coulomb cap holds",
                       "for (int k = 0; k < 3; k++) dt_new[k] = -(Ft[k] + eta_t * vt[k]) / kt;",
                       ";"),
    "vt_drop_spin": ("Eq. 4: tangential velocity includes the spin term",
                     "vt[k] = G->v[k] - vn[k] + sxn[k];",
                     "vt[k] = G->v[k] - vn[k];"),
    "hertz_radius": ("Eqs. 8-9: Hertz stiffness from the effective radius",
                     "double q = sqrt(G->delta * G->R);",
                     "double q = sqrt(G->delta * G->R * 2.0);"),
    "inertia": ("solid-sphere moment of inertia 2/5 m r^2",
                "s->I[i] = 0.4 * s->m[i] * ri * ri;",
                "s->I[i] = 0.5 * s->m[i] * ri * ri;"),
    "wall_mass": ("Sec. 4.2 Step 8: a wall is a particle of infinite mass",
                  "    G->M = s->m[a];\n    return ORC_OK;\n}",
                  "    G->M = 0.5 * s->m[a];\n    return ORC_OK;\n}"),
    "contact_le": ("contact means d < r_i + r_j",
                   "return d2 < S * S;",
                   "return d2 <= S * S * 1.000001;"),
    "stencil_2d": ("Eq. 12: 27 cells, not 9",
                   "for (int dz = -1; dz <= 1; dz++)",
                   "for (int dz = 0; dz <= 0; dz++)"),
    "kick_gravity": ("KDK kick with the external field",
                     "s->v[3 * i + k] += h * (s->F[3 * i + k] / s->m[i] + s->p.g[k]);",
                     "s->v[3 * i + k] += h * (s->F[3 * i + k] / s->m[i] + 2*s->p.g[k]);"),
    "simple_sign": ("Eq. 1: damping opposes the relative velocity",
                    "F[k] = -p->k_sp * G->delta * G->n[k] - p->k_da * G->v[k] - p->k_sh * vts[k];",
                    "F[k] = -p->k_sp * G->delta * G->n[k] + p->k_da * G->v[k] - p->k_sh * vts[k];"),
    "simple_shear_sign": ("Eq. 1: the shear term opposes the tangential velocity",
                          "- p->k_sh * vts[k];",
                          "+ p->k_sh * vts[k];"),
    "simple_shear_dropped": ("Eq. 1: the shear term k_sh v_t is part of the force",
                             "- p->k_sh * vts[k];",
                             ";"),
    "simple_shear_spin": ("Eq. 1: v_t is the tangential part of v, with no spin term",
                          "vts[k] = G->v[k] - vn[k];",
                          "vts[k] = G->v[k] - vn[k] + sxn[k];"),
    "rotational_ke_mass": ("rotational kinetic energy I |w|^2 / 2",
                           "term[4] = 0.5 * s->I[i] * dot3(w, w);",
                           "term[4] = 0.5 * s->m[i] * dot3(w, w);"),
    "hertz_energy_factor": ("Eqs. 8-9: Hertz elastic energy (2/5) K delta^(5/2)",
                            "en = 0.4 * K.kn * sqrt(G.R) * pow(G.delta, 2.5)",
                            "en = 0.5 * K.kn * sqrt(G.R) * pow(G.delta, 2.5)"),
    "tangential_energy_dropped": ("Eq. 4: tangential spring energy k_t |delta_t|^2 / 2",
                                  "en = 0.5 * kn * G.delta * G.delta + 0.5 * kt * dot3(h, h);",
                                  "en = 0.5 * kn * G.delta * G.delta;"),
    "material_self": ("Eqs. 8-10: the constants of the pair (i, j), not of i alone",
                      "int32_t ta = s->type[a], tb = b >= 0 ? s->type[b] : s->wall_type;",
                      "int32_t ta = s->type[a], tb = ta;"),
    "material_wall": ("Step 8: a wall has its own material",
                      "int32_t ta = s->type[a], tb = b >= 0 ? s->type[b] : s->wall_type;",
                      "int32_t ta = s->type[a], tb = b >= 0 ? s->type[b] : 0;"),
    "material_ignored": ("Eqs. 8-10: a material-pair table replaces the single material",
                         "if (s->ntypes == 0) {",
                         "if (1) {"),
    "material_alpha": ("Eq. 10: alpha of the pair's restitution",
                       "mat[q].alpha = alpha_of(table[4 * q + 2]);",
                       "mat[q].alpha = s->alpha;"),
    "material_mu": ("Eq. 5: the pair's friction coefficient",
                    "mat[q].mu = table[4 * q + 3];",
                    "mat[q].mu = s->p.mu;"),
    "cohesion_sign": ("cohesion pulls the bodies together",
                      "F[k] += p->cohesion * G->n[k];",
                      "F[k] -= p->cohesion * G->n[k];"),
    "rolling_sign": ("rolling resistance opposes the relative spin",
                     "C[k] = -p->rolling_mu * G->R * fn * G->wrel[k] / wn;",
                     "C[k] = p->rolling_mu * G->R * fn * G->wrel[k] / wn;"),
    "rolling_partner_sign": ("the rolling couple acts on the partner in the opposite sense",
                             "T[3 * b + q] += s->r[b] * nxft[q] - Cr[q];",
                             "T[3 * b + q] += s->r[b] * nxft[q] + Cr[q];"),
    "rolling_lever": ("the rolling couple's lever arm is the effective radius",
                      "C[k] = -p->rolling_mu * G->R * fn * G->wrel[k] / wn;",
                      "C[k] = -p->rolling_mu * 2.0 * G->R * fn * G->wrel[k] / wn;"),
    "rolling_total_normal": ("the rolling couple scales with Eq. 4's |F_n|, not the net normal force",
                             "C[k] = -p->rolling_mu * G->R * fn * G->wrel[k] / wn;",
                             "C[k] = -p->rolling_mu * G->R * fabs(dot3(F, G->n)) * G->wrel[k] / wn;"),
    "plate_unbounded": ("a plate is finite: its nearest point is clamped to the rectangle",
                        "q[u] = c[u] < P->lo[0] ? P->lo[0] : (c[u] > P->hi[0] ? P->hi[0] : c[u]);",
                        "q[u] = c[u];"),
    "plate_normal_sign": ("n points from the centre to the plate's nearest point",
                          "G->n[k] = -d[k] / dist;",
                          "G->n[k] = d[k] / dist;"),
    "plate_index": ("wall w >= 6 is plate w - 6",
                    "plate_nearest(&s->p.plates[w - 6], s->x + 3 * a, q, d);\n        return",
                    "plate_nearest(&s->p.plates[w == 6 ? 1 : 0], s->x + 3 * a, q, d);\n        return"),
    "history_side": ("Eq. 6: the history seen from the other particle is negated",
                     "const double *h = he ? he->d : zero;",
                     "double hneg[3]; if (he) { hneg[0]=-he->d[0]; hneg[1]=-he->d[1]; hneg[2]=-he->d[2]; } "
                     "const double *h = he ? (b >= 0 && (a ^ b) & 1 ? hneg : he->d) : zero;"),
}

PINS = os.path.join(ROOT, "tests", "test_oracle_pins.py")
SLOW = "tests/test_oracle_pins.py::test_energy_drift_plain_fp64_workload"


def _build(src_text, out_dir, name):
    c = os.path.join(out_dir, f"{name}.c")
    lib = os.path.join(out_dir, f"lib_{name}.so")
    with open(c, "w") as f:
        f.write(src_text)
    subprocess.run(["gcc", "-O3", "-std=c99", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared", c,
                    "-o", lib, "-lm"], check=True, capture_output=True)
    return lib


def _pins_against(lib):
    env = dict(os.environ, DEM_ORACLE_LIB=lib)
    r = subprocess.run([sys.executable, "-m", "pytest", PINS, "-q", "-x", "-p", "no:cacheprovider",
                        "--deselect", SLOW], env=env, capture_output=True, text=True, cwd=ROOT, timeout=300)
    tail = (r.stdout.strip().splitlines() or [""])[-1]
    return r.returncode, tail


def test_every_planted_mistake_fails_a_pin(tmp_path):
    src = open(SRC).read()
    for name, (_, old, _new) in MUTATIONS.items():
        assert src.count(old) >= 1, f"mutation {name}: its text is no longer in the oracle source"

    def run(item):
        name, (_, old, new) = item
        lib = _build(src.replace(old, new, 1), str(tmp_path), name)
        return name, _pins_against(lib)

    control = _pins_against(_build(src, str(tmp_path), "control"))
    assert control[0] == 0, f"the unchanged source fails its pins: {control[1]}"
    with ThreadPoolExecutor(max_workers=4) as ex:
        results = dict(ex.map(run, MUTATIONS.items()))
    # exit status 1: tests ran and at least one failed (not a crash or a usage error)
    missed = {n: t for n, (rc, t) in results.items() if rc != 1}
    assert not missed, f"mistakes no pin caught (or that crashed the run): {missed}"
