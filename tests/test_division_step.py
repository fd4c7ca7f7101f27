"""The tile sweep divides a centroid sum by its neighbour count with a
reciprocal table and one correction step instead of a full division, for
sums of magnitude at least 128 x the smallest normal number (smaller ones,
zero included, are divided).  This checks on the host (C, libm's fma) that
the step gives the correctly rounded quotient for every count 1..127, in
double and float, over random values of every exponent and values whose
quotient lies beside a rounding boundary -- and that the bound is needed:
below it, where a quotient can be subnormal, the step does go wrong.  The
GPU parity tests check the kernel itself against the oracle."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))


def test_division_by_count_is_correctly_rounded(tmp_path):
    exe = str(tmp_path / "div_step")
    subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-o", exe,
                           os.path.join(HERE, "cdiv", "div_step.c"), "-lm"])
    out = subprocess.check_output([exe, "100000"], text=True).split()
    stepped, bad, below_bad = int(out[0]), int(out[1]), int(out[2])
    assert stepped > 127 * 100000      # most doubles and floats of the sample are above the bound
    assert bad == 0
    assert below_bad > 0
