"""GPU parity: the HIP qdot path against the CPU oracle, through the C ABI.

Integer outputs (exponent histogram, per-component classes, counts, e_min,
e_max, N_bins, t, flags) must match bit for bit.  The value must be within
1e-13 * sum_i |x_i y_i| of the oracle's value; the bound within a relative
1e-12 (it is an FP64 sum taken in a different order).
"""
from __future__ import annotations

import json
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle
import workloads

torch = pytest.importorskip("torch")
import paper_2105_00115_amd as q  # noqa: E402

pytestmark = pytest.mark.gpu

VALUE_TOL = 1e-13
GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "worked_examples.json")


@pytest.fixture(scope="module")
def h():
    handle = q.Qdot(0)
    yield handle
    handle.close()


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to("cuda:0")


def compare(h, x, y, tol, opt=None, xd=None, yd=None, check_classes=True):
    xd = dev(x) if xd is None else xd
    yd = dev(y) if yd is None else yd
    cls, hist, r = h.qdot_classes(xd, yd, tol, opt=opt)
    o = oracle.qdot(x, y, tol, opt=opt, want_classes=True, want_hist=True)
    assert r["status"] == o["status"]
    if o["status"] != oracle.OK:
        return r, o
    for k in ("count", "n_zero", "e_min", "e_max", "n_bins", "t", "flags"):
        assert r[k] == o[k], (k, r[k], o[k])
    np.testing.assert_array_equal(hist.cpu().numpy(), o["hist"])
    if check_classes:
        np.testing.assert_array_equal(cls.cpu().numpy(), o["classes"])
    scale = oracle.abs_dot(x, y)
    assert abs(r["value"] - o["value"]) <= VALUE_TOL * scale, (r["value"], o["value"], scale)
    for c in range(3):
        assert abs(r["part"][c] - o["part"][c]) <= VALUE_TOL * scale
    assert abs(r["bound_rel"] - o["bound_rel"]) <= 1e-12 * abs(o["bound_rel"])
    # the synchronous entry point gives the same result as the debug one
    r2 = h.qdot(xd, yd, tol, opt=opt)
    assert r2["count"] == r["count"] and r2["value"] == r["value"]
    return r, o


def _golden_inputs(case):
    if "x" in case:
        x = np.array([float.fromhex(s) for s in case["x"]])
        y = np.array([float.fromhex(s) for s in case["y"]])
        return x, y, float(case["tol"])
    if "ones" in case:
        n = case["ones"]
        return np.ones(n), np.ones(n), float(case["tol"])
    n = 4160
    x = np.zeros(n)
    y = np.ones(n)
    x[0] = 1.0
    x[64:4158] = 2.0 ** -24
    if case["name"] == "tile_tree_rounds":
        x[1] = x[3] = 2.0 ** -24
    else:
        x[2] = x[3] = 2.0 ** -24
    return x, y, 2.0 ** -20


@pytest.mark.parametrize("name", [c["name"] for c in json.load(open(GOLDEN))["cases"]])
def test_golden_examples_exact(h, name):
    case = next(c for c in json.load(open(GOLDEN))["cases"] if c["name"] == name)
    x, y, tol = _golden_inputs(case)
    r, o = compare(h, x, y, tol)
    v = case["expect"].get("value")
    if v is not None:
        want = eval(v.replace("2**", "Fraction(2)**"), {"Fraction": Fraction}) \
            if isinstance(v, str) else Fraction(v)
        assert Fraction(r["value"]) == want


@pytest.mark.parametrize("tol", [1e-3, 1e-6, 1e-10])
@pytest.mark.parametrize("seed", [1, 2])
def test_c1_law_n1e5(h, tol, seed):
    x, y = workloads.log_uniform_pair(100000, seed)
    compare(h, x, y, tol)


@pytest.mark.parametrize("n", [0, 1, 2, 3, 5, 63, 64, 65, 255, 256, 257, 1023, 1024, 1025,
                               4097, 65537, 100003])
def test_ragged_lengths(h, n):
    x, y = workloads.log_uniform_pair(n, 100 + n)
    compare(h, x, y, 1e-6)


@pytest.mark.parametrize("off", [1, 3])
def test_unaligned_views(h, off):
    # 8-byte but not 16-byte aligned vectors take the scalar-load path; tiles
    # still start at the first element of the view
    n = 50001
    x, y = workloads.log_uniform_pair(n + off, 7)
    xd, yd = dev(x), dev(y)
    compare(h, x[off:], y[off:], 1e-6, xd=xd[off:], yd=yd[off:])
    compare(h, x[off:], y[1:n + 1], 1e-6, xd=xd[off:], yd=yd[1:n + 1])


@pytest.mark.parametrize("opt", [[1, 0, 0, 0], [0, 1, 0, 0], [0, 0, 1, 0], [1, 1, 1, 0]])
def test_options(h, opt):
    x, y = workloads.log_uniform_pair(60000, 9)
    compare(h, x, y, 1e-6, opt=opt)


@pytest.mark.parametrize("law,t", [("A", 20), ("A", 100), ("B", 6), ("B", 30)])
def test_paper_distributions(h, law, t):
    gen = workloads.paper_dist_a if law == "A" else workloads.paper_dist_b
    x, y = gen(70000, t, 11)
    for tol in (1e-16, 1e-8, 1e-3):
        compare(h, x, y, tol)


def test_edge_cases(h):
    # all zero products
    r, o = compare(h, np.zeros(1000), np.ones(1000), 1e-6)
    assert r["value"] == 0.0 and r["flags"] & q.F_ALL_PERF
    # mixed zeros
    x, y = workloads.log_uniform_pair(5000, 12)
    x[::3] = 0.0
    y[::7] = -0.0
    compare(h, x, y, 1e-6)
    # subnormal operands (both exponent paths)
    g = workloads.rng(13)
    x = np.ldexp(g.uniform(1, 2, 3000), g.integers(-1074, -1000, 3000))
    y = np.ldexp(g.uniform(-2, 2, 3000), g.integers(900, 1000, 3000))
    compare(h, x, y, 1e-9)
    # huge and tiny tolerances
    x, y = workloads.log_uniform_pair(5000, 14)
    r, _ = compare(h, x, y, 1e300)
    assert r["value"] == 0.0 and r["count"][q.PERF] == 5000
    r, _ = compare(h, x, y, 1e-300)
    assert r["count"][q.DOUBLE] == 5000
    # single element
    compare(h, np.array([3.0]), np.array([-0.5]), 1e-6)


def test_empty_inputs(h):
    # n = 0: +0 with no bins, in every mode and entry point, as the oracle
    e = torch.zeros(0, dtype=torch.float64, device="cuda:0")
    z = np.zeros(0)
    keys = ("count", "n_zero", "e_min", "e_max", "n_bins", "t", "flags", "status", "passes",
            "e_ref")
    for opt in (None, [0, 0, 0, 1], [0, 0, 0, 0, 1]):
        r = h.qdot(e, e, 1e-6, opt=opt)
        o = oracle.qdot(z, z, 1e-6, opt=opt)
        for k in keys:
            assert r[k] == o[k], (opt, k, r[k], o[k])
        assert r["value"] == 0.0 and not np.signbit(r["value"])
    cls, hist, r = h.qdot_classes(e, e, 1e-6)
    assert cls.numel() == 0 and int(hist.abs().sum()) == 0 and r["n_bins"] == 0
    ef = torch.zeros(0, dtype=torch.float32, device="cuda:0")
    rf = h.qdot_f32(ef, ef, 1e-6)
    of = oracle.qdot_f32(np.zeros(0, dtype=np.float32), np.zeros(0, dtype=np.float32), 1e-6)
    for k in keys:
        assert rf[k] == of[k], k
    assert h.fp64_dot(e, e) == 0.0


def test_nonfinite_and_bad_arguments(h):
    x, y = workloads.log_uniform_pair(3000, 15)
    for bad in (np.nan, np.inf, -np.inf):
        xb = x.copy()
        xb[1234] = bad
        r = h.qdot(dev(xb), dev(y), 1e-6)
        assert r["status"] == q.E_NONFINITE and np.isnan(r["value"])
        # the oracle's error result field for field: every other field 0
        o = oracle.qdot(xb, y, 1e-6)
        for k in ("count", "n_zero", "e_min", "e_max", "n_bins", "t", "flags", "status",
                  "bound_rel", "bound_abs", "lower", "e_ref", "passes"):
            assert r[k] == o[k], (k, r[k], o[k])
        assert r["part"] == [0.0, 0.0, 0.0]
    # the workspace recovers: the next call is normal
    compare(h, x, y, 1e-6)
    for tol in (0.0, -1.0, float("nan"), float("inf")):
        with pytest.raises(q.QdotError):
            h.qdot(dev(x), dev(y), tol)
    with pytest.raises(q.QdotError):
        h.qdot(dev(x), dev(y), 1e-6, opt=[3, 0, 0, 0])


def test_repeat_and_tuning_invariance(h):
    x, y = workloads.log_uniform_pair(300000, 16)
    xd, yd = dev(x), dev(y)
    base_cls, base_hist, base = h.qdot_classes(xd, yd, 1e-6)
    again = h.qdot(xd, yd, 1e-6)
    assert again["value"] == base["value"]  # same launch configuration: bitwise
    o = oracle.qdot(x, y, 1e-6)
    scale = oracle.abs_dot(x, y)
    # launch shapes, both forms of the accumulate pass, histogram copies,
    # threads per block
    for sb, su, ab, au, af, hc, nt in [(1, 1, 1, 1, 0, 8, 256), (2, 2, 8, 4, 1, 8, 512),
                                       (8, 4, 2, 2, 1, 1, 128), (16, 1, 16, 2, 0, 2, 512),
                                       (4, 2, 1, 4, 1, 4, 256), (2, 1, 2, 2, 1, 8, 128),
                                       (1, 4, 1, 1, 0, 8, 512)]:
        h.set_tune(-1, sb, su, ab, au, 4, 1, af, hc, nt)
        cls, hist, r = h.qdot_classes(xd, yd, 1e-6)
        assert torch.equal(cls, base_cls) and torch.equal(hist, base_hist)
        assert r["count"] == base["count"]
        assert abs(r["value"] - o["value"]) <= VALUE_TOL * scale
    h.reset_tune()


def test_tune_file_loading(h, tmp_path):
    good = tmp_path / "good.txt"
    good.write_text("# comment\n0 1 1 2 2\n3 8 4 16 1  # trailing comment\n2 1 2 4 4 8 2\n"
                    "1 2 1 2 2 4 1 1 4\n\n")
    h.reset_tune()
    d0 = h.get_tune(0)
    d2 = h.get_tune(2)
    h.load_tune(str(good))
    # a 5-column line leaves the one-pass shape and the rest as they were
    assert h.get_tune(0) == (1, 1, 2, 2) + d0[4:] and h.get_tune(3)[:4] == (8, 4, 16, 1)
    assert h.get_tune(2) == (1, 2, 4, 4, 8, 2) + d2[6:]
    assert h.get_tune(1) == (2, 1, 2, 2, 4, 1, 1, 4, 256)
    wide = tmp_path / "wide.txt"
    wide.write_text("3 2 1 2 2 4 1 0 8 512\n")
    h.load_tune(str(wide))
    assert h.get_tune(3) == (2, 1, 2, 2, 4, 1, 0, 8, 512)
    # the solver line sets the solver and batched launch shapes
    solver = tmp_path / "solver.txt"
    solver.write_text("solver 2 65536 8192 32 4 1 1\n")
    h.load_tune(str(solver))
    assert h.get_solver_tune() == (2, 65536, 8192, 32, 4, 1, 1)
    for line in ("solver 2 65536 8192\n", "solver 2 65536 8192 32 4 3 0\n",
                 "solver 2 65536 8192 32 4 1 2\n"):
        solver.write_text(line)
        with pytest.raises(q.QdotError):
            h.load_tune(str(solver))
    assert h.get_solver_tune() == (2, 65536, 8192, 32, 4, 1, 1)
    h.set_solver_tune()
    for line in ("1 2 3 4 5\n",            # unroll 3 is not allowed
                 "1 2 1 2 2 4 1 2 8\n",    # acc_form 2
                 "1 2 1 2 2 4 1 0 3\n",    # 3 histogram copies
                 "1 2 1 2 2 4 1 0\n",      # 8 columns
                 "1 2 1 2 2 4 1 0 8 384\n"):  # 384 threads per block
        bad = tmp_path / "bad.txt"
        bad.write_text(line)
        with pytest.raises(q.QdotError):
            h.load_tune(str(bad))
    assert h.get_tune(1) == h.get_tune(1)  # unchanged, still readable
    with pytest.raises(q.QdotError):
        h.load_tune(str(tmp_path / "missing.txt"))
    h.reset_tune()


def test_async_result_in_stream_order(h):
    x, y = workloads.log_uniform_pair(20000, 17)
    xd, yd = dev(x), dev(y)
    outs = torch.zeros(3 * q.RESULT_BYTES, dtype=torch.uint8, device="cuda:0")
    base = outs.data_ptr()
    for i, tol in enumerate((1e-3, 1e-6, 1e-10)):
        h.qdot_async(xd, yd, tol, base + i * q.RESULT_BYTES)
    torch.cuda.synchronize()
    for res, tol in zip(q.parse_results(outs), (1e-3, 1e-6, 1e-10)):
        o = oracle.qdot(x, y, tol)
        assert res["count"] == o["count"] and res["t"] == o["t"]


@pytest.mark.parametrize("mode", [0, 1])
def test_graph_replay_of_one_call(h, mode):
    # no memset nodes: the workspace is reset by the kernels themselves
    opt = [0, 0, 0, mode]
    x, y = workloads.log_uniform_pair(300001, 20)
    xd, yd = dev(x), dev(y)
    eager = torch.zeros(q.RESULT_BYTES, dtype=torch.uint8, device="cuda:0")
    h.qdot_async(xd, yd, 1e-6, eager, opt=opt)
    torch.cuda.synchronize()
    out = torch.zeros_like(eager)
    st = torch.cuda.Stream()
    st.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.stream(st):
        with torch.cuda.graph(g, stream=st):
            h.qdot_async(xd, yd, 1e-6, out, opt=opt)
    torch.cuda.synchronize()
    for rep in range(4):
        out.zero_()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(out, eager), rep
        h.qdot(xd[:7000], yd[:7000], 1e-3, opt=opt)  # eager work on the same handle
        torch.cuda.synchronize()
    o = oracle.qdot(x, y, 1e-6, opt=opt)
    r = q.parse_results(out)[0]
    assert r["count"] == o["count"]
    assert abs(r["value"] - o["value"]) <= VALUE_TOL * oracle.abs_dot(x, y)


def test_minimal_entry_point(h):
    x, y = workloads.log_uniform_pair(50000, 19)
    xd, yd = dev(x), dev(y)
    v, counts = q.qdot_simple(xd, yd, 1e-6)
    r = h.qdot(xd, yd, 1e-6)
    assert counts == r["count"]
    o = oracle.qdot(x, y, 1e-6)
    assert counts == o["count"]
    # its own handle may use another launch shape: FP64 reduction order only
    assert abs(v - o["value"]) <= VALUE_TOL * oracle.abs_dot(x, y)
    with pytest.raises(q.QdotError):
        q.qdot_simple(xd, yd, -1.0)


def test_fp64_dot_baseline(h):
    x, y = workloads.log_uniform_pair(1 << 20, 18)
    d = h.fp64_dot(dev(x), dev(y))
    exact = oracle.dot_exact(x, y)
    # recursive summation bound: |err| <= gamma_n * sum |x_i y_i|
    assert abs(d - exact) <= 1e-10 * oracle.abs_dot(x, y)


def test_binding_before_torch_in_a_fresh_process():
    # a script that creates a handle before it imports torch itself: torch's
    # HIP runtime must still be the one the process uses
    import subprocess
    import sys
    code = ("import paper_2105_00115_amd as q\n"
            "h = q.Qdot(0)\n"
            "import torch\n"
            "x = torch.ones(1000, dtype=torch.float64, device='cuda:0')\n"
            "r = h.qdot(x, x, 1e-6)\n"
            "assert r['value'] == 1000.0, r\n"
            "print('ok')\n")
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    p = subprocess.run([sys.executable, "-c", code], cwd=root, capture_output=True, text=True,
                       timeout=240)
    assert p.returncode == 0 and p.stdout.strip().endswith("ok"), p.stderr[-2000:]


def test_device_info(h):
    dev, cus = h.device_info()
    assert dev == 0 and cus == torch.cuda.get_device_properties(0).multi_processor_count


def test_timing_api(h):
    x, y = workloads.log_uniform_pair(1 << 20, 90)
    xd, yd = dev(x), dev(y)
    h.timing_read()  # start from an empty record
    h.timing_enable(True)
    for _ in range(3):
        h.qdot(xd, yd, 1e-6)
    for _ in range(2):
        h.fp64_dot(xd, yd)
    t = h.timing_read()
    h.timing_enable(False)
    assert t["qdot_calls"] == 3 and t["dot64_calls"] == 2
    assert t["scan_ms"] > 0 and t["acc_ms"] > 0 and t["dot64_ms"] > 0
    assert t["cut_ms"] >= 0 and t["fin_ms"] >= 0
    # read clears the record; calls while disabled are not timed
    h.qdot(xd, yd, 1e-6)
    t2 = h.timing_read()
    assert t2["qdot_calls"] == 0 and t2["dot64_calls"] == 0 and t2["scan_ms"] == 0.0


def test_autotuner_on_small_buckets(tmp_path):
    # a short sweep of the two smallest buckets: every swept shape (grid,
    # groups in flight, both accumulate forms, 1/2/4/8 histogram copies, the
    # one-pass grid) must reproduce the reference classes and histogram bit
    # for bit (the tuner compares them and raises otherwise), the file must
    # load back, and the tuned handle must give the same counts as the
    # defaults
    from paper_2105_00115_amd import autotune
    handle, chosen, checked = autotune.tune(reps=2, buckets=[0, 1], log=lambda m: None)
    path = str(tmp_path / "tune.txt")
    autotune.write(path, chosen, "gfx950", handle.device_info()[1],
                   batch=(4, 131072, 16384, 16, 8, 2, 0))
    handle.close()
    assert [c[0] for c in chosen] == [0, 1]
    # per bucket: 15 grid shapes, up to 1 mixed, 23 form/copies/threads
    # shapes, 1 final
    assert checked >= 2 * (15 + 23 + 1)
    for c in chosen:
        assert c[2][6] in autotune.ACC_FORM and c[2][7] in autotune.HIST_COPIES
        assert c[2][8] in autotune.BLOCK_THREADS
    with q.Qdot(0, load_tuned=False) as tuned, q.Qdot(0, load_tuned=False) as plain:
        tuned.load_tune(path)
        for n in (30000, 500000):
            x, y = workloads.log_uniform_pair(n, 91)
            a = tuned.qdot(dev(x), dev(y), 1e-6)
            b = plain.qdot(dev(x), dev(y), 1e-6)
            assert a["count"] == b["count"] and a["flags"] == b["flags"]
            assert abs(a["value"] - b["value"]) <= VALUE_TOL * oracle.abs_dot(x, y)
