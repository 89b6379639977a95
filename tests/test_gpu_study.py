"""The accuracy-study harness (paper_2406_11751_amd.study) on a reduced sweep:
the paper's Section 5.1 claims on its coherent test matrices with smoothing --
residual below 1e-15 for every sampling amount, orthogonality below 1e-12 from
c = 2n on, the Section 5.2 estimate 4 eps kappa(A1) within a small factor, and
Lemma l_31 on the smoothed sample of Q."""
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def test_reduced_accuracy_study():
    from paper_2406_11751_amd import study

    print("case: reduced accuracy study (m = 6000, n = 100 .. 300, kappa = 1e15)", flush=True)
    rep = study.main(["--quick", "--trials", "3"])
    for c, row in rep["sweep_c"]["100"].items():
        s = row["summary"]
        c = int(c)
        if c >= 200:
            assert s["failures"] == 0
            assert s["orth"]["max"] < 1e-12
        if "orth" in s:
            assert s["residual"]["max"] < 1e-15
            assert 0.02 < s["orth_over_estimate"]["min"] and s["orth_over_estimate"]["max"] < 20
        if c >= 200:
            assert row["lemma_l31_rel_dev_kappa1e6"] < 1e-7
    for n, s in rep["sweep_n"].items():
        assert s["failures"] == 0 and s["orth"]["max"] < 1e-12 and s["residual"]["max"] < 1e-15
