"""The oracle's pins are not vacuous: plausible mistakes, planted one at a
time in a scratch copy of ``oracle/lbm_oracle.c`` (under pytest's temporary
directory; the oracle itself is untouched), each make the pins named beside
them fail.

The mistakes are the kind a reader of the paper could make: the printed sign
of the eighth source entry of Eq. 8 (reading R2), a sign or component slip in
a y-term (advection, divergence, gravity, plate adhesion of Eq. 14), the
bounce-back partner of the diagonal links, a dropped factor in the
pseudopotential of Eq. 10 or in the nine-point Laplacian, the full instead of
the half force in the velocity of Eq. 13, and a mistyped row of the matrix M
of Eq. 6.
"""
import importlib.util
import os
import shutil

import pytest

import test_oracle_eos as TE
import test_oracle_flows as TF
import test_oracle_lattice as TL
import test_oracle_symmetry as TS
import test_oracle_thermal as TT

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ORACLE_PY = os.path.join(ROOT, "oracle", "oracle.py")
ORACLE_C = os.path.join(ROOT, "oracle", "lbm_oracle.c")

pytestmark = pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")


def _yref(m):
    TS.test_step_commutes_with_y_reflection(m, 0.0)


MUTANTS = {
    "Eq8-S8-printed-sign": ("S[8] = ux * Fy + uy * Fx;", "S[8] = ux * Fy - uy * Fx;",
                            [lambda m: TL.test_bgk_guo_special_case(m, 1.0),
                             TS.test_step_commutes_with_transpose_on_periodic_box]),
    "advection-y-sign": ("out[c] = -(s->ux[c] * tx + s->uy[c] * ty)",
                         "out[c] = -(s->ux[c] * tx - s->uy[c] * ty)",
                         [TT.test_advection_term_exact_on_linear_field,
                          TS.test_step_commutes_with_transpose_on_periodic_box]),
    "adhesion-sign": ("double Fay = -p->Gw * s->psi[c] * p->psiw * swy;",
                      "double Fay = p->Gw * s->psi[c] * p->psiw * swy;",
                      [TF.test_force_assembly_closed_form_at_plates]),
    "divergence-y-uses-ex": ("div += w * (EX[i] * uxn + EY[i] * uyn);",
                             "div += w * (EX[i] * uxn + EX[i] * uyn);",
                             [TT.test_compression_term_on_linear_velocity, _yref]),
    "gravity-component": ("double Fby = (r - p->rho_v) * p->gy;",
                          "double Fby = (r - p->rho_v) * p->gx;",
                          [TF.test_force_assembly_closed_form_at_plates,
                           TS.test_step_commutes_with_x_reflection]),
    "bounce-back-mirror": ("static const int OPP[9] = {0, 3, 4, 1, 2, 7, 8, 5, 6};",
                           "static const int OPP[9] = {0, 3, 4, 1, 2, 8, 7, 6, 5};",
                           [lambda m: TF.test_poiseuille_exact_with_magic_rates(m, 1.0)]),
    "psi-factor-2": ("double arg = 2.0 * (orc_peos(p, rho, T) - rho / 3.0) / p->G;",
                     "double arg = (orc_peos(p, rho, T) - rho / 3.0) / p->G;",
                     [TE.test_psi_reproduces_eos_pressure]),
    "laplacian-factor-2": ("lap += 2.0 * w * (Tn - Ts[c]);", "lap += w * (Tn - Ts[c]);",
                           [TT.test_conduction_term_exact_on_quadratic_field]),
    "full-force-velocity": ("s->ux[c] = (jx + 0.5 * s->Fx[c]) / r;",
                            "s->ux[c] = (jx + s->Fx[c]) / r;",
                            [lambda m: TF.test_poiseuille_exact_with_magic_rates(m, 1.0),
                             TS.test_step_commutes_with_transpose_on_periodic_box]),
    "M-row-8": ("{0, 0, 0, 0, 0, 1, -1, 1, -1}};", "{0, 0, 0, 0, 0, 1, 1, -1, -1}};",
                [TL.test_M_rows_are_lallemand_luo_moments]),
}


def _mutant_oracle(name, old, new, tmp_path):
    src = open(ORACLE_C).read()
    assert src.count(old) == 1, "mutation site not found (oracle source changed?): " + name
    c_path = tmp_path / "lbm_oracle_mutant.c"
    c_path.write_text(src.replace(old, new))
    spec = importlib.util.spec_from_file_location("oracle_mutant", ORACLE_PY)
    m = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(m)
    m.SRC = str(c_path)
    m.LIB = str(tmp_path / "liblbm_oracle_mutant.so")
    m.build(force=True)
    return m


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_planted_mistake_fails_its_pins(name, tmp_path):
    old, new, pins = MUTANTS[name]
    m = _mutant_oracle(name, old, new, tmp_path)
    for pin in pins:
        with pytest.raises(AssertionError):
            pin(m)


def test_unmutated_copy_passes_the_same_pins(orc, tmp_path):
    """The scratch-copy route itself changes nothing: the oracle's own
    source, loaded the same way, passes every pin used above."""
    m = _mutant_oracle("identity", "static const int OPP[9]", "static const int OPP[9]", tmp_path)
    seen = set()
    for _, _, pins in MUTANTS.values():
        for pin in pins:
            if id(pin) not in seen:
                seen.add(id(pin))
                pin(m)
