"""Batched runs (one persistent launch per heavy phase over several runs) against the same runs
stepped one at a time, and one of them against the FP64 oracle.  Batched and single results
differ only by the order of floating-point atomic additions."""
import numpy as np
import pytest

import pic_inputs as pi
from oracle import Oracle

gpu = pytest.mark.gpu
NAMES = ["Ex", "Ey", "Ez", "Bx", "By", "Bz", "Jx", "Jy", "Jz"]


def _workloads():
    a = pi.small_boosted(real="f32", nx=40, nz=150, ppc=2)
    b = pi.small_boosted(real="f32", nx=33, nz=121, ppc=3, seed=91, gamma=5.0)
    c = pi.small_lab(real="f32", nx=24, nz=96, ppc=4)
    return [a, b, c]


def _scales(w):
    from test_gpu_parity import field_scales
    return field_scales(Oracle.from_workload(w))


def _max_err(sa, sb, w):
    sc = _scales(w)
    out = {}
    for n in NAMES:
        fa, fb = sa.field(n), sb.field(n)
        s = max(np.abs(fa).max(), sc[n[0]])
        out[n] = float(np.abs(fa - fb).max() / s) if s > 0 else float(np.abs(fa - fb).max())
    return out


@gpu
def test_batch_equals_single_runs():
    from paper_1009_2727_amd import Batch, Sim
    ws = _workloads()
    singles = [Sim.from_workload(w, sort_every=7) for w in ws]
    batched = [Sim.from_workload(w, sort_every=7) for w in ws]
    for s in singles:
        s.step(45)
    b = Batch(batched)
    b.step(45)
    for w, s1, s2 in zip(ws, singles, batched):
        assert s2.sync_status() == 0
        errs = _max_err(s1, s2, w)
        assert max(errs.values()) <= 2e-6, errs
        assert np.array_equal(s1.counts(), s2.counts())


@gpu
def test_batched_run_matches_oracle():
    from paper_1009_2727_amd import Batch, Sim
    from test_gpu_parity import compare_fields
    ws = _workloads()
    sims = [Sim.from_workload(w) for w in ws]
    Batch(sims).step(30)
    ref = Oracle.from_workload(ws[0])
    ref.step(30)
    compare_fields(sims[0], ref, 1e-5, tag="batched boosted f32")


@gpu
def test_batch_with_learned_filter_and_single_steps_between():
    from paper_1009_2727_amd import Batch, Sim, bilinear_factor_params
    ws = _workloads()[:2]
    w2 = pi.copy_workload(ws[1])
    w2["config"]["filter_kind"] = 1
    single = [Sim.from_workload(ws[0]), Sim.from_workload(ws[1])]
    batched = [Sim.from_workload(ws[0]), Sim.from_workload(w2)]
    batched[1].set_learned_filter(bilinear_factor_params(4, True))
    single[0].step(20)
    single[1].step(17)
    b = Batch(batched)
    b.step(10)
    batched[0].step(3)          # a run's own steps interleave with the batch
    b.step(7)
    for w, s1, s2 in zip(ws, single, batched):
        errs = _max_err(s1, s2, w)
        assert max(errs.values()) <= 1e-5, errs


@gpu
def test_batch_with_strided_filter_equals_single_runs():
    # a batch now runs each run's own line filter, so strided filters batch too
    from paper_1009_2727_amd import Batch, Sim
    ws = _workloads()[:2]
    ws[1]["config"]["filter_strides"] = 0x3      # S(1:2)
    singles = [Sim.from_workload(w, sort_every=7) for w in ws]
    batched = [Sim.from_workload(w, sort_every=7) for w in ws]
    for s in singles:
        s.step(30)
    Batch(batched).step(30)
    for w, s1, s2 in zip(ws, singles, batched):
        assert s2.sync_status() == 0
        errs = _max_err(s1, s2, w)
        assert max(errs.values()) <= 2e-6, errs
