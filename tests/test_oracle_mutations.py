"""Planted mistakes: each plausible slip in the oracle must fail at least one pin.

Every mutation edits a private copy of the oracle's C source (on the CPU, in a
temporary directory), builds it with the oracle's own flags, and runs the
quick pins against that build.  The real oracle is untouched.
"""

import os
import subprocess

import pytest

import oracle
import pins
from oracle.build import CFLAGS, SRC

MUTATIONS = {
    "dissipation sign": ("- alpha * 0.5 * (QR[k] - QL[k])", "+ alpha * 0.5 * (QR[k] - QL[k])"),
    "alpha from velocity difference": ("fabs(0.5 * (unL + unR))", "fabs(0.5 * (unL - unR))"),
    "alpha without sound speed": ("+ 0.5 * (cL + cR);", "+ 0.0 * (cL + cR);"),
    "pressure dropped from momentum flux": ("rL * unL * unL + pL", "rL * unL * unL"),
    "pressure dropped from energy flux": ("(UL[3] + pL) * unL", "UL[3] * unL"),
    "rotation back uses wrong tangent component": ("len * (Fp[1] * ex + Fp[2] * tx)",
                                                  "len * (Fp[1] * ex + Fp[2] * ty)"),
    "tangential momentum flux sign": ("rL * unL * vtL", "-rL * unL * vtL"),
    "face length not applied": ("Fout[0] = len * Fp[0];", "Fout[0] = Fp[0];"),
    "normal not normalised": ("double ex = nx / len, ey = ny / len;", "double ex = nx, ey = ny;"),
    "sound speed without gamma": ("*c = sqrt(gamma * (*p) / (*rho));", "*c = sqrt((*p) / (*rho));"),
    "kinetic energy without one half": ("U[3] - 0.5 * (*rho)", "U[3] - 1.0 * (*rho)"),
    "update sign": ("cur[4 * i + k] - coef * R[k]", "cur[4 * i + k] + coef * R[k]"),
    "area multiplies instead of divides": ("double coef = dt / area[i];", "double coef = dt * area[i];"),
    "neighbour of the wrong face": ("int64_t j = nbr[3 * i + f];", "int64_t j = nbr[3 * i + (f + 1) % 3];"),
    "normal components swapped": ("nrm[6 * i + 2 * f], nrm[6 * i + 2 * f + 1]",
                                  "nrm[6 * i + 2 * f + 1], nrm[6 * i + 2 * f]"),
    "in-place update (reads new values)": ("double *cur = U, *nxt = Un;", "double *cur = U, *nxt = U;"),
    "children in descending id order": ("(bd == kd && kid[b] > key)", "(bd == kd && kid[b] < key)"),
    "root not moved to the far end": ("if (ecc_x > ecc_r) {", "if (ecc_x > ecc_r + 1000000) {"),
    "S_BW from prefix minimum": ("if (s[i + 1] < s[i])\n            s[i] = s[i + 1];",
                                 "if (s[i + 1] > s[i])\n            s[i] = s[i + 1];"),
    "bandwidth not doubled": ("out[1] = 2 * B + 1;", "out[1] = B + 1;"),
    "AM1 ties go to the larger id": ("(score == best_score && k < best)",
                                     "(score == best_score && k > best)"),
    "AM1 scores node(I) too": ("if (p >= 0 && knb[g] != vI)", "if (p >= 0)"),
    "exact S_BW counts the union with repeats": ("if (pos[kn[g]] < 0 && seen[kn[g]] != m) {",
                                                 "if (pos[kn[g]] < 0) {"),
    "exact S_BW without s(i)": ("exact_out[m] = (size - 1 - m) + un + sv[m];",
                                "exact_out[m] = (size - 1 - m) + un;"),
    "bounded pattern ignores its stop rule": ("if (max_imp > bound && I > 0)",
                                              "if (max_imp > bound + 1000000 && I > 0)"),
    "bounded pattern executes node(I) too": ("const int run = k < I && !ghost[k];",
                                             "const int run = k <= I && !ghost[k];"),
}


@pytest.fixture(scope="module")
def source():
    with open(SRC) as f:
        return f.read()


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_mutant_is_caught(name, source, tmp_path):
    old, new = MUTATIONS[name]
    assert source.count(old) == 1, f"mutation site for '{name}' must occur exactly once"
    src = tmp_path / "mutant.c"
    src.write_text(source.replace(old, new))
    lib = str(tmp_path / "libmutant.so")
    subprocess.run(["gcc", *CFLAGS, str(src), "-o", lib, "-lm"], check=True)
    o = oracle.Oracle(lib)
    failed = []
    for pin in pins.QUICK_PINS:
        try:
            ok, _ = pin(o)
        except Exception:  # a crash or a non-finite result also counts as caught
            ok = False
        if not ok:
            failed.append(pin.__name__)
    assert failed, f"mutation '{name}' passed every pin"
