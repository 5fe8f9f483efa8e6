"""The seeded input generators: determinism and the ranges of the workloads
they stand in for (host only)."""
import math

import numpy as np

import scp_inputs as si

TWO_PI = 2 * math.pi


def test_generators_are_deterministic():
    a, b = si.config5(), si.config5()
    assert [m["EJ"] for m in a["modes"]] == [m["EJ"] for m in b["modes"]]
    assert [c["g"] for c in a["couplings"]] == [c["g"] for c in b["couplings"]]
    r1, r2 = si.serving_request(17), si.serving_request(17)
    assert r1["n_steps"] == r2["n_steps"] and r1["want_grad"] == r2["want_grad"]
    assert np.array_equal(si.poisson_arrivals(50, 2.0), si.poisson_arrivals(50, 2.0))


def test_config_shapes():
    c1, c3, c5 = si.config1(), si.config3(), si.config5()
    assert [m["trunc"] for m in c1["modes"]] == [4, 4] and c1["n_steps"] == 2000
    assert len(c1["columns"]) == 16
    assert [m["trunc"] for m in c3["modes"]] == [5] * 4 and c3["n_steps"] == 5000
    assert len(c3["columns"]) == 16
    # 2 channels x 20 Gaussian-basis amplitudes
    assert sum(len(d["params"]) for d in c3["drives"]) == 40
    assert [m["trunc"] for m in c5["modes"]] == [3] * 8 and len(c5["columns"]) == 256
    assert len(c5["couplings"]) == 8 and len(c5["drives"]) == 8
    for m in c5["modes"]:
        ec = m["EC"] / TWO_PI
        assert 0.2 <= ec <= 0.3 and 40 <= m["EJ"] / m["EC"] <= 60
    for c in c5["couplings"]:
        assert 5e-3 <= c["g"] / TWO_PI <= 15e-3


def test_serving_requests_follow_the_mix():
    fams, grads = set(), 0
    for r in range(200):
        q = si.serving_request(r)
        n = len(q["modes"])
        d = q["modes"][0]["trunc"]
        assert 2 <= n <= 6 and d in (3, 4, 5) and d ** n <= 3125
        assert 20.0 <= q["T"] <= 200.0 and q["n_steps"] == round(50 * q["T"])
        assert len(q["columns"]) == 2 ** n
        fams.add(q["family"])
        grads += bool(q["want_grad"])
    assert len(fams) == 3
    assert 60 <= grads <= 140
