"""GPU parity of the batched ragged 1-D stepper against the FP64 CPU oracle:
every instance must equal the oracle run of its own 1 x 1 x L lattice, and the
persistent launch, its HIP graph and the one-launch-per-instance schedule must
agree bit for bit.  The MM scheme in difference form ("mmd") is checked
against the oracle of the full MM scheme, whose E and B it reproduces."""
import numpy as np
import pytest
import torch

import oracle
from paper_2309_08068_amd import inputs, lbem
from parity import check, floor_bounds, rel

pytestmark = pytest.mark.gpu


def oracle_instance(model, eps, mu, sig, E0, B0, steps, real="f64"):
    L = len(eps)
    P = oracle.Problem("mm" if model == "mmd" else model, (1, 1, L), eps_r=eps, mu_r=mu, sigma=sig)
    f = oracle.init(P, E0, B0, real=real)
    oracle.run(P, f, 0, steps)
    E, B, _, _ = oracle.fields(P, f, steps)
    return E, B


def random_batch(seed, lengths):
    rng = np.random.default_rng(seed)
    off = np.concatenate([[0], np.cumsum(lengths)]).astype(np.int64)
    tot = int(off[-1])
    return dict(off=off, eps=rng.uniform(1, 3, tot), mu=rng.uniform(1, 2, tot), sig=rng.uniform(0, 0.2, tot),
                E0=rng.normal(size=(3, tot)), B0=rng.normal(size=(3, tot)))


@pytest.mark.parametrize("model", ["mm", "hv", "mmd"])
@pytest.mark.parametrize("storage", ["f32"])
def test_batch_random_parity_and_schedules(model, storage):
    lengths = [1, 2, 3, 17, 64, 65, 255, 256, 257, 700, 1031, 5]
    d = random_batch(42, lengths)
    steps = 9
    outs = {}
    for sched in ("persistent", "graph", "per_instance"):
        b = lbem.Batch(model, d["off"], d["eps"], d["mu"], d["sig"], storage=storage)
        b.set_launch(128, 1)
        b.set_fields(d["E0"], d["B0"])
        if sched == "persistent":
            b.step(4)
            b.step(5)
        elif sched == "graph":
            b.step_graph(4)
            b.step_graph(5)
        else:
            b.step_per_instance(9)
        assert b.time == steps
        E, B = b.fields()
        torch.cuda.synchronize()
        outs[sched] = (E.cpu().numpy(), B.cpu().numpy())
    for sched in ("graph", "per_instance"):
        assert np.array_equal(outs[sched][0], outs["persistent"][0]), sched
        assert np.array_equal(outs[sched][1], outs["persistent"][1]), sched
    E, B = (x.astype(np.float64) for x in outs["persistent"])
    for i in range(len(lengths)):
        s, e = d["off"][i], d["off"][i + 1]
        Eo, Bo = oracle_instance(model, d["eps"][s:e], d["mu"][s:e], d["sig"][s:e], d["E0"][:, s:e], d["B0"][:, s:e],
                                 steps)
        check(E[:, s:e], Eo, what=f"instance {i} E")
        check(B[:, s:e], Bo, what=f"instance {i} B")


def test_batch_autotune_leaves_state_unchanged():
    d = random_batch(7, [300, 5000, 1200, 64] * 8)
    b = lbem.Batch("mm", d["off"], d["eps"], d["mu"], d["sig"])
    b.set_fields(d["E0"], d["B0"])
    b.step(3)
    E0, _ = b.fields()
    E0 = E0.clone()
    threads, gpc = b.autotune(4)
    assert threads in (128, 256, 512, 1024) and gpc >= 1
    assert b.time == 3
    E1, _ = b.fields()
    assert torch.equal(E0, E1)


@pytest.mark.parametrize("model", ["mm", "mmd"])
def test_multilayer_workload_sampled_parity(model):
    """The full multilayer workload (512 instances, lengths 500..8000, 5000
    steps) in the autotuned launch configuration the benchmark times; the
    shortest, the longest and two random instances are compared with the
    oracle run of each instance.  MM only: HV grows an interface mode at
    every layer boundary (see the oracle's spectral test)."""
    bt = inputs.multilayer("mm", steps=5000)
    b = lbem.batch_from_inputs(bt, model=model)
    b.autotune(10)
    b.step(bt.steps)
    E, B = b.fields()
    E = E.double().cpu().numpy()
    B = B.double().cpu().numpy()
    L = bt.lengths
    rng = np.random.default_rng(3)
    pick = {int(np.argmin(L)), int(np.argmax(L)), *map(int, rng.choice(len(L), 2, replace=False))}
    for i in sorted(pick):
        w = bt.instance(i)
        Eo, Bo = oracle_instance(model, w.eps_r, w.mu_r, w.sigma, w.E0, w.B0, bt.steps)
        Ef, Bf = oracle_instance(model, w.eps_r, w.mu_r, w.sigma, w.E0, w.B0, bt.steps, real="f32")
        tol, etol, fr, fe = floor_bounds((Ef, Bf), (Eo, Bo))
        s, e = bt.offsets[i], bt.offsets[i + 1]
        eE = check(E[:, s:e], Eo, tol, etol, f"instance {i} E")
        eB = check(B[:, s:e], Bo, tol, etol, f"instance {i} B")
        print(f"instance {i} (L={e - s}): float32 floor {fr:.2e} (element-wise {fe:.2e}), GPU error "
              f"E {eE[0]:.2e} / {eE[1]:.2e}, B {eB[0]:.2e} / {eB[1]:.2e}", flush=True)


def test_batch_rejects_bad_offsets_and_media():
    with pytest.raises(lbem.LbemError):
        lbem.Batch("mm", [0, 5, 5, 9])
    with pytest.raises(lbem.LbemError):
        lbem.Batch("mm", [1, 5])
    with pytest.raises(lbem.LbemError) as e:
        lbem.Batch("mm", [0, 4], eps_r=np.full(4, 0.5))
    assert e.value.status == -4


TB_LENGTHS = [1, 2, 3, 17, 255, 256, 257, 300, 511, 512, 513, 700, 1031, 2000, 5003]


@pytest.mark.parametrize("model", ["mm", "hv", "mmd"])
@pytest.mark.parametrize("storage", ["f32", "bf16", "f16"])
def test_temporal_blocking_is_bit_identical(model, storage):
    """Temporally blocked passes (resident instances up to one workgroup of
    cells, trapezoidal tiles with LDS-kept halos beyond) give the bits of one
    step per pass, for every tile width and pass length, with odd first and
    last steps, a last tile narrower than the halo, and the graph path."""
    d = random_batch(77, TB_LENGTHS)
    calls = (5, 16, 3, 40, 1, 2)

    def run(threads, gpc, k, graph=False):
        b = lbem.Batch(model, d["off"], d["eps"], d["mu"], d["sig"], storage=storage)
        b.set_launch(threads, gpc)
        b.set_blocking(k)
        assert b.blocking() == k
        b.set_fields(d["E0"], d["B0"])
        for n in calls:
            (b.step_graph if graph else b.step)(n)
        assert b.time == sum(calls)
        E, B = b.fields()
        torch.cuda.synchronize()
        return E.clone(), B.clone()

    ref = run(256, 2, 0)
    assert torch.isfinite(ref[0]).all()
    for threads, gpc, k, graph in ((256, 1, 2, False), (256, 2, 8, False), (256, 1, 16, False), (512, 1, 8, False),
                                   (512, 1, 32, False), (512, 1, 64, False), (512, 1, 16, True), (256, 2, 32, True),
                                   (256, 1, 64, False), (1024, 1, 32, False), (1024, 1, 64, True)):
        out = run(threads, gpc, k, graph)
        print(f"{model} {storage} threads {threads} k {k} graph {graph}: identical "
              f"{torch.equal(out[0], ref[0]) and torch.equal(out[1], ref[1])}", flush=True)
        assert torch.equal(out[0], ref[0]) and torch.equal(out[1], ref[1]), (threads, gpc, k, graph)


def test_temporal_blocking_matches_oracle_and_autotune():
    """A blocked run against the oracle instance by instance, and the
    autotuner (which also tries blocked passes) leaving the state unchanged."""
    lengths = [40, 511, 1500, 3001]
    d = random_batch(5, lengths)
    b = lbem.Batch("mm", d["off"], d["eps"], d["mu"], d["sig"])
    b.set_launch(512, 1)
    b.set_blocking(16)
    b.set_fields(d["E0"], d["B0"])
    b.step(3)
    E0 = b.fields()[0].clone()
    threads, gpc = b.autotune(4)
    k = b.blocking()
    assert k in (0, 16, 32, 48, 64) and (k == 0 or threads in (256, 512, 1024))
    assert b.time == 3 and torch.equal(b.fields()[0], E0)
    b.step(36)
    E, B = (x.double().cpu().numpy() for x in b.fields())
    for i in range(len(lengths)):
        s, e = d["off"][i], d["off"][i + 1]
        Eo, Bo = oracle_instance("mm", d["eps"][s:e], d["mu"][s:e], d["sig"][s:e], d["E0"][:, s:e],
                                 d["B0"][:, s:e], 39)
        check(E[:, s:e], Eo, what=f"instance {i} E")
        check(B[:, s:e], Bo, what=f"instance {i} B")


def test_temporal_blocking_rejects_bad_settings():
    b = lbem.Batch("hv", [0, 10, 30])
    for k in (1, 3, 35, 66, -2):
        with pytest.raises(lbem.LbemError):
            b.set_blocking(k)
    b.set_launch(128, 4)
    with pytest.raises(lbem.LbemError):
        b.set_blocking(8)
    b.set_launch(512, 1)
    b.set_blocking(8)
    with pytest.raises(lbem.LbemError):
        b.set_launch(128, 4)
    assert b.blocking() == 8
