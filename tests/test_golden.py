"""The oracle against the closed-form values stored in tests/golden/
closed_forms.txt (each line names its passage; written by
tests/golden/make_closed_forms.py from textbook formulas, no renderer code).
The scenes are stored as FP32, as every renderer input is, so the comparison
allows the relative rounding of FP32 inputs (1e-6)."""
import os

import numpy as np
import pytest

import oracle
import helpers as H
from paper_2412_03378_amd import scenes

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _rows():
    out = []
    for line in open(os.path.join(GOLDEN, "closed_forms.txt")):
        if line.startswith("#") or not line.strip():
            continue
        name, inputs, value, cite = [f.strip() for f in line.split("|")]
        kw = {k: float(v) for k, v in (item.split("=") for item in inputs.split())}
        out.append((name, kw, float(value), cite))
    return out


ROWS = _rows()


def test_fixture_matches_its_generator():
    import runpy
    gen = runpy.run_path(os.path.join(GOLDEN, "make_closed_forms.py"))
    assert open(os.path.join(GOLDEN, "closed_forms.txt")).read() == gen["text"]()


def _axis_cam(distance, f, size=65, znear=0.2):
    c = (size) / 2.0
    return scenes.Camera(np.eye(3, dtype=np.float32), np.float32([0, 0, distance]), f, f, c, c,
                         size, size, znear=znear)


@pytest.mark.parametrize("name,kw,value,cite", ROWS, ids=[f"{r[0]}-{i}" for i, r in enumerate(ROWS)])
def test_oracle_matches_closed_form(name, kw, value, cite):
    c = 32                                   # centre pixel of a 65-pixel axis camera
    if name in ("iso_x", "iso_alpha"):
        s = kw["s"]
        sc = H.scene([[kw["r_over_s"] * s, 0.0, 0.0]], [s] * 3, kw["kappa"])
        st = oracle.Settings.no_thresholds(mode="xray")
        x = oracle.render(sc, _axis_cam(4.0, 100.0), st, pixels=[(c, c)])["image"][0, 0]
        got = x if name == "iso_x" else -np.expm1(-x)
    elif name == "theta_x":
        sc = H.scene([[0.0, 0.0, 0.0]], [0.07] * 3, kw["theta"])
        st = oracle.Settings.no_thresholds(mode="xray", density="theta")
        got = oracle.render(sc, _axis_cam(4.0, 100.0), st, pixels=[(c, c)])["image"][0, 0]
    elif name == "near_x":
        sc = H.scene([[0.0, 0.0, 0.0]], [kw["s"]] * 3, kw["kappa"])
        st = oracle.Settings.no_thresholds(mode="xray", near_segment=True)
        cam = _axis_cam(kw["z0"], 100.0, znear=kw["zn"])
        got = oracle.render(sc, cam, st, pixels=[(c, c)])["image"][0, 0]
    elif name == "splat_alpha":
        sc = H.scene([[0.0, 0.0, 0.0]], [kw["s"]] * 3, kw["o"], rgb=[[1.0, 1.0, 1.0]])
        st = oracle.Settings(alpha_min=1e-30, alpha_max=1.0 - 1e-12, T_min=0.0,
                             alpha_model="splat")
        cam = _axis_cam(kw["z"], kw["f"])
        got = oracle.render(sc, cam, st, pixels=[(c + int(kw["r"]), c)])["image"][0, 0]
    elif name == "epan_x":
        s = kw["s"]
        sc = H.scene([[kw["r_over_s"] * s, 0.0, 0.0]], [s] * 3, kw["kappa"])
        st = oracle.Settings.no_thresholds(mode="xray", kernel="epanechnikov")
        got = oracle.render(sc, _axis_cam(4.0, 100.0), st, pixels=[(c, c)])["image"][0, 0]
        if value == 0.0:   # outside the support (up to the rounding of D^2 = 1)
            assert abs(got) < 1e-20, cite
            return
    else:
        pytest.fail(f"unknown row {name}")
    assert got == pytest.approx(value, rel=1e-6), cite
