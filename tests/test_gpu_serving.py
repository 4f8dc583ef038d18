"""GPU tests of the serving loop (continuous batching): every request gets the
coefficients of a single call on the same inputs, whatever it was batched
with ("alone vs mix"), in the precision the FP64-fallback rule gives it; the
HBM budget bounds what is in flight; latencies are recorded."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _pool(n_meshes=5, seed=11):
    from paper_2107_10942_amd import serving
    from q2x_inputs import configs
    rng = np.random.default_rng(seed)
    return [serving.pinned_mesh(configs.serving_job(rng, nmin=3e3, nmax=6e4)) for _ in range(n_meshes)]


def _requests(pool, n, rate, seed):
    from paper_2107_10942_amd import serving
    rng = np.random.default_rng(seed)
    arr = serving.poisson_arrivals(n, rate, rng)
    reqs = []
    for i in range(n):
        mi = int(rng.integers(0, len(pool)))
        reqs.append(serving.Request(kind=int(rng.integers(0, 2)), p=int(rng.integers(8, 25)), arrival=float(arr[i]),
                                    mesh_id=mi, **pool[mi]))
    return reqs


def _alone(r):
    import torch
    from paper_2107_10942_amd import q2x
    t = [x.cuda() for x in (r.verts, r.elems, r.density, r.elem_box, r.box_center)]
    o = q2x.run(r.kind, *t, None, r.p, precision=r.precision)
    torch.cuda.synchronize()
    return o


@pytest.mark.parametrize("resident", [True, False])
@pytest.mark.parametrize("budget_mb", [4096, 24])
def test_serving_alone_vs_mix(budget_mb, resident):
    """Alone vs in the mix, with meshes kept resident in HBM (requests on a
    resident mesh skip the upload; the small budget forces evictions) and
    with every mesh uploaded per request; two compute streams."""
    import torch
    from paper_2107_10942_amd import q2x, serving
    pool = _pool()
    reqs = _requests(pool, 40, rate=4000.0, seed=3)
    srv = serving.Server(torch.device("cuda:0"), hbm_budget=budget_mb << 20, max_batch=8, p_fp32_max=16,
                         keep_outputs=True, resident=resident, compute_streams=2)
    srv.serve(reqs)
    summ = serving.latency_summary(reqs)
    print(budget_mb, resident, srv.stats, {k: round(v, 3) if isinstance(v, float) else v for k, v in summ.items()},
          flush=True)
    assert all(r.done > 0 for r in reqs)
    assert summ["p50_ms"] > 0 and summ["p99_ms"] >= summ["p50_ms"]
    sizes = np.bincount([r.batch for r in reqs])
    if budget_mb == 24:
        assert srv.stats["batches"] > len(reqs) // 8  # the budget split the bursts
    if resident and budget_mb == 4096:
        # five meshes: each uploaded once, every later request on it a hit
        assert srv.stats["uploads"] == len({r.mesh_id for r in reqs})
        assert summ["resident_hit_rate"] > 0.8
    if not resident:
        assert srv.stats["resident_hits"] == 0 and srv.stats["resident_meshes"] == 0
    for r in reqs:
        assert r.precision == (q2x.FP64 if r.p > 16 else q2x.FP32_MIXED)
        assert torch.equal(r.out, _alone(r)), (r.kind, r.p, r.batch, sizes[r.batch])
