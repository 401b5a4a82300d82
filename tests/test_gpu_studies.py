"""The synthetic studies of Sec. 4.1 on the device: the driver at a small
scale, and the library against the oracle on the studies' own inputs."""
from __future__ import annotations

import json

import numpy as np
import pytest

import oracle
import workloads

torch = pytest.importorskip("torch")
import paper_2105_00115_amd as q  # noqa: E402
from paper_2105_00115_amd import studies  # noqa: E402

pytestmark = pytest.mark.gpu

VALUE_TOL = 1e-13


@pytest.fixture(scope="module")
def h():
    handle = q.Qdot(0)
    yield handle
    handle.close()


@pytest.mark.parametrize("family,t", [("A", 10), ("A", 100), ("B", 2), ("B", 30), ("B", 13)])
@pytest.mark.parametrize("eps", [1e-16, 1e-6, 1e-1])
def test_study_inputs_match_the_oracle(h, family, t, eps):
    print(f"[gpu-case] study family={family} t={t} eps={eps}", flush=True)
    xd, yd = workloads.paper_dist_torch(20000, t, 5000 + t, family)
    x, y = xd.cpu().numpy(), yd.cpu().numpy()
    # the law: s * 2^p with s in [0.5, 1) (both families are positive)
    m, _ = np.frexp(x)
    assert (m >= 0.5).all() and (m < 1.0).all()
    r = h.qdot(xd, yd, eps)
    o = oracle.qdot(x, y, eps)
    for k in ("count", "n_zero", "e_min", "e_max", "n_bins", "t", "flags", "status"):
        assert r[k] == o[k], k
    assert abs(r["value"] - o["value"]) <= VALUE_TOL * oracle.abs_dot(x, y)
    # positive products: Thm 3.3's hypothesis holds, and the error against
    # the exact dot stays within the bound
    ex = oracle.dot_exact(x, y)
    assert abs(r["value"] - ex) <= r["bound_rel"] * abs(ex)


def test_small_studies(tmp_path):
    out = tmp_path / "studies.json"
    assert studies.main(["--study", "all", "--scale", "small", "--out", str(out)]) == 0
    d = json.load(open(out))
    e1 = d["e1"]["cells"]
    assert {(c["family"], c["n"]) for c in e1} == {(f, n) for f in "AB" for n in (100, 1000)}
    for c in e1:
        assert c["bad_status"] == 0 and c["samples"] > 0
        assert np.isfinite(c["bound_minus_relerr"]["median"])
    e2 = d["e2"]
    assert len(e2["cells"]) == 2 * 3 * 2 * len(e2["eps"])
    for c in e2["cells"]:
        # effectiveness: relerr against the FP64 dot stays below the tolerance
        assert c["relerr_max"] <= c["eps"]
        assert abs(sum(c["class_frac_mean"]) - 1.0) < 1e-5  # stored to 6 digits
    for c in e2["timing"]:
        assert c["calls"] > 0 and 0.0 < c["approx_efficiency"] < 1.0
