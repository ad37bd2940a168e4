"""The autotuner (dade_autotune) on the GPU: it reports every configuration it timed, picks the
fastest one that meets the agreement bound, its agreement is what a plain search with the chosen
options gives, the chosen options' results match the oracle run with the same Delta_d and round
shape, and the launch shape it tunes leaves results bitwise unchanged."""
import numpy as np
import pytest

from oracle import ivf
from paper_2411_17229_amd import dade, workloads
from gpu_helpers import artifacts, compare, oracle_ivf, oracle_index, to_np

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def env():
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    w = workloads.WORKLOADS["small-20k-d128"]
    X, Q = workloads.make(w, n_queries=300)
    oi, _, _ = oracle_index(X, w.nlist, w.seed, alpha=w.alpha)
    gi = dade.dade_import(artifacts(oi), torch.from_numpy(X).cuda())
    return dict(w=w, X=X, Q=Q, Qd=torch.from_numpy(Q).cuda(), oi=oi, gi=gi)


def agreement(env, ids, K, nprobe):
    ref, _ = dade.dade_search(env["gi"], env["Qd"], K, nprobe, mode="full_d")
    ref = to_np(ref)
    a = [len(set(ids[q][ids[q] >= 0].tolist()) & set(ref[q][ref[q] >= 0].tolist())) / max(1, (ref[q] >= 0).sum())
         for q in range(len(ids))]
    return float(np.mean(a))


def test_autotune_picks_the_fastest_agreeing_configuration(env):
    w = env["w"]
    chosen, table = dade.dade_autotune(env["gi"], env["Qd"], w.k, w.nprobe, min_agreement=0.9, reps=3)
    n_grid = 5 * 3   # Delta_d {8..128} x 3 round shapes, then 2 launch shapes
    assert len(table) == n_grid + 2
    grid = table[:n_grid]
    assert {t["delta_d"] for t in grid} == {8, 16, 32, 64, 128}
    ok = [t for t in grid if t["agreement"] >= 0.9]
    assert ok, grid
    fastest = min(ok, key=lambda t: t["ms"])
    for key in ("delta_d", "schedule", "fill_min", "growth"):
        assert chosen[key] == fastest[key], (chosen, fastest)
    # the launch-shape step keeps the winner's agreement
    for t in table[n_grid:]:
        assert t["delta_d"] == fastest["delta_d"] and t["agreement"] == fastest["agreement"]
    # the reported agreement is a plain search's with the chosen options
    ids, _ = dade.dade_search(env["gi"], env["Qd"], w.k, w.nprobe, **chosen)
    assert abs(agreement(env, to_np(ids), w.k, w.nprobe) - fastest["agreement"]) < 1e-6


def test_chosen_options_match_the_oracle(env):
    w = env["w"]
    chosen, _ = dade.dade_autotune(env["gi"], env["Qd"], w.k, w.nprobe, min_agreement=0.9, reps=2)
    ids, d2 = dade.dade_search(env["gi"], env["Qd"], w.k, w.nprobe, **chosen)
    torch.cuda.synchronize()
    o = oracle_ivf(env["oi"], env["Q"], w.k, w.nprobe, chosen["delta_d"],
                   schedule=chosen["schedule"], fill_min=chosen["fill_min"], growth=chosen["growth"])
    compare(o, to_np(ids), to_np(d2), env["X"], env["Q"], w.k)


def test_launch_shape_does_not_change_results(env):
    w = env["w"]
    kw = dict(delta_d=32, schedule="doubling", fill_min=32, growth=0)
    base_ids, base_d2 = dade.dade_search(env["gi"], env["Qd"], w.k, w.nprobe, **kw)
    base_ids, base_d2 = to_np(base_ids), to_np(base_d2)
    for bpc in (1, 2, 3, 64):
        ids, d2 = dade.dade_search(env["gi"], env["Qd"], w.k, w.nprobe, scan_blocks_per_cu=bpc, **kw)
        assert np.array_equal(to_np(ids), base_ids), bpc
        assert np.array_equal(to_np(d2).view(np.uint32), base_d2.view(np.uint32)), bpc


def test_autotune_uneven_batch(env):
    """Per-query K and nprobe (the uneven-batch workload's form): the tuner runs on them and an
    impossible agreement bound falls back to the most agreeing configuration."""
    w = env["w"]
    K, npb = workloads.uneven_batch(len(env["Q"]), 1, 40, (1, 10, 50, 100), seed=4)
    kp, npp = torch.from_numpy(K).cuda(), torch.from_numpy(npb).cuda()
    chosen, table = dade.dade_autotune(env["gi"], env["Qd"], 100, 40, k_per_query=kp, nprobe_per_query=npp,
                                       min_agreement=1.0, reps=2)
    grid = table[:15]
    if not any(t["agreement"] >= 1.0 for t in grid):
        best = max(t["agreement"] for t in grid)
        assert [t for t in grid if t["delta_d"] == chosen["delta_d"] and t["schedule"] == chosen["schedule"]
                and t["growth"] == chosen["growth"]][0]["agreement"] == best
    o = oracle_ivf(env["oi"], env["Q"], K, np.minimum(npb, w.nlist), chosen["delta_d"],
                   schedule=chosen["schedule"], fill_min=chosen["fill_min"], growth=chosen["growth"])
    ids, d2 = dade.dade_search(env["gi"], env["Qd"], 100, 40, k_per_query=kp, nprobe_per_query=npp, **chosen)
    torch.cuda.synchronize()
    compare(o, to_np(ids), to_np(d2), env["X"], env["Q"], K)


def test_autotune_argument_errors(env):
    w = env["w"]
    with pytest.raises(dade.DadeError):
        dade.dade_autotune(env["gi"], env["Qd"], w.k, w.nprobe, min_agreement=1.5)
    with pytest.raises(dade.DadeError):
        dade.dade_autotune(env["gi"], env["Qd"], w.k, w.nprobe, mode="full_d")
