"""GPU tests of the batched persistent launches (include/xrt_batch.h): parity
with the FP64 oracle (same 1e-5 relative-L2 gate as single plans), agreement
with single plans, results independent of the launch configuration (every
line sum and every tile gather is done by one workgroup), HIP graph replays
equal to eager runs, and the autotuner."""
import math

import numpy as np
import pytest
import torch

import oracle
import xrt_workloads as W

pytestmark = pytest.mark.gpu


def rel(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


@pytest.fixture(scope="module")
def mixed():
    """Thirteen problems: sizes 1x1 .. 130x70, degrees 0-3 and the box spline,
    parallel, fan, random lines."""
    from paper_2503_20907_amd import batch, ops
    rng = np.random.default_rng(71)
    probs = []
    shapes = [(64, 64, 1), (130, 70, 3), (48, 100, 0), (96, 96, 2), (128, 128, 3), (1, 1, 1), (33, 17, 3),
              (64, 80, 1), (100, 64, 3), (20, 20, 0), (128, 96, 2), (72, 56, oracle.BOX3), (50, 50, oracle.BOX3)]
    for i, (nx, ny, n) in enumerate(shapes):
        kind = i % 3
        N = max(nx, ny)
        if kind == 0:
            spec = W.parallel_beam(int(rng.integers(10, 60)), int(math.ceil(1.5 * N)) + 2)
        elif kind == 1:
            spec = W.fan_beam(int(rng.integers(10, 50)), int(math.ceil(1.5 * N)), 2.0 * N + 4, N, n)
        else:
            spec = W.random_lines(int(rng.integers(200, 3000)), N, seed=100 + i)
        c = rng.normal(size=(ny, nx)).astype(np.float32)
        probs.append({"nx": nx, "ny": ny, "n": n, "spec": spec, "c": c, "lc": oracle.lines(spec)})
    b = batch.Batch([(p["nx"], p["ny"], p["n"], ops.Lines.from_spec(p["spec"])) for p in probs])
    for k, p in enumerate(probs):
        b.coeffs(k).copy_(torch.as_tensor(p["c"], device="cuda"))
    yield b, probs
    b.close()


def outputs(b):
    torch.cuda.synchronize()
    return [(b.sino(k).cpu().numpy().copy(), b.back(k).cpu().numpy().copy()) for k in range(len(b))]


def test_batch_matches_oracle(mixed):
    b, probs = mixed
    b.forward()
    b.adjoint()
    out = outputs(b)
    for k, p in enumerate(probs):
        print(f"problem {k}: {p['nx']}x{p['ny']} degree {p['n']}", flush=True)
        s_ref = oracle.forward(p["n"], p["c"].astype(np.float64), p["lc"])
        if np.linalg.norm(s_ref) > 0:
            assert rel(out[k][0], s_ref) < 1e-5, k
        b_ref = oracle.adjoint(p["n"], out[k][0].astype(np.float64), p["lc"], p["nx"], p["ny"])
        if np.linalg.norm(b_ref) > 0:
            assert rel(out[k][1], b_ref) < 1e-5, k
        # adjoint identity <H c, s> = <c, H^T s> with s the batch's own sinogram
        lhs = float(np.dot(out[k][0].astype(np.float64), out[k][0].astype(np.float64)))
        rhs = float(np.sum(p["c"].astype(np.float64) * out[k][1].astype(np.float64)))
        if lhs > 0:
            assert abs(lhs - rhs) <= 1e-5 * lhs, k


def test_batch_matches_single_plans(mixed):
    from paper_2503_20907_amd import ops
    b, probs = mixed
    b.forward()
    b.adjoint()
    out = outputs(b)
    for k, p in enumerate(probs):
        plan = ops.Plan(p["nx"], p["ny"], p["n"], ops.Lines.from_spec(p["spec"]))
        s1 = plan.forward(torch.as_tensor(p["c"], device="cuda"))
        a1 = plan.adjoint(torch.as_tensor(out[k][0], device="cuda")).cpu().numpy()
        s1 = s1.cpu().numpy()
        if np.linalg.norm(s1) > 0:
            assert rel(out[k][0], s1) < 2e-6, k
        if np.linalg.norm(a1) > 0:
            assert rel(out[k][1], a1) < 2e-6, k
        plan.close()


def test_results_do_not_depend_on_configuration(mixed):
    b, probs = mixed
    ref = None
    for cfg in [(4, 256, 2), (1, 2048, 1), (16, 512, 8), (2, 1024, 4)]:
        b.set_config(*cfg)
        b.forward()
        b.adjoint()
        out = outputs(b)
        if ref is None:
            ref = out
            continue
        for k in range(len(probs)):
            assert np.array_equal(out[k][0], ref[k][0]) and np.array_equal(out[k][1], ref[k][1]), (cfg, k)
    b.set_config(4, 256, 2)


def test_graph_replays_equal_eager(mixed):
    b, probs = mixed
    b.run(graph=False)
    eager = outputs(b)
    for rep in range(3):
        # eager work and synchronisation between replays; clear the outputs first
        for k in range(len(probs)):
            b.sino(k).fill_(-1.0)
            b.back(k).fill_(-1.0)
        torch.cuda.synchronize()
        b.run(graph=True)
        out = outputs(b)
        for k in range(len(probs)):
            assert np.array_equal(out[k][0], eager[k][0]) and np.array_equal(out[k][1], eager[k][1]), (rep, k)


def test_autotune_keeps_results(mixed):
    b, probs = mixed
    b.forward()
    b.adjoint()
    before = outputs(b)
    cfg = b.autotune(reps=1)
    assert cfg["lines_per_item"] in (256, 512, 1024, 2048)
    assert 1 <= cfg["fwd_blocks_per_cu"] <= 32 and 1 <= cfg["adj_blocks_per_cu"] <= 32
    assert b.config == cfg
    b.forward()
    b.adjoint()
    after = outputs(b)
    for k in range(len(probs)):
        assert np.array_equal(after[k][0], before[k][0]) and np.array_equal(after[k][1], before[k][1])
    info = b.info()
    assert info["adjoint_items"] > 0 and info["forward_items"] > 0
