"""Batched persistent wavefront (many jobs of uneven size sharing one path
pool, hipGraph-captured iterations): every job's image must match the
oracle's image of that job (its job index keys the random numbers) and
equal, bit for bit, the same job rendered alone."""
import numpy as np
import pytest

from paper_2605_27323_amd import scenes
from tests._parity import assert_parity, oracle_image

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2605_27323_amd import ptmi  # noqa: E402


def log(*a):
    print(*a, flush=True)


def _jobs(with_scenes=False):
    specs = [(1000, 8, 33, 21, 2), (1001, 40, 64, 48, 3), (1002, 3, 40, 8, 1), (1003, 15, 17, 29, 4)]
    Rs, args, sc = [], [], []
    for j, (seed, n, w, h, spp) in enumerate(specs):
        s, c = scenes.procedural(seed=seed, n_objects=n, width=w, height=h)
        Rs.append(ptmi.Renderer(s, c))
        args.append(dict(spp=spp, max_depth=6, rr_start=3, seed=5, frame=1))
        sc.append((s, c))
    return (Rs, args, sc) if with_scenes else (Rs, args)


def _oracle_check(imgs, args, sc, what):
    # job j != 0 keys the random numbers with j: the oracle renders job j
    # from its own scene copy with the same key
    for j, ((s, c), kw) in enumerate(zip(sc, args)):
        ref, frag, _ = oracle_image(s, c, job=j, **{k: v for k, v in kw.items() if k != "sampler"},
                                    sampler=1 if kw.get("sampler") == "halton" else 0)
        assert_parity(imgs[j].cpu().numpy(), ref, frag, what=f"{what} job {j}")


@pytest.mark.parametrize("capacity,graph,iters,pools", [(0, True, 0, 0), (256, True, 4, 1), (1000, False, 0, 1),
                                                        (64, True, 16, 1), (0, True, 0, 2), (256, True, 4, 4),
                                                        (1000, False, 0, 3)])
def test_batch_equals_standalone(capacity, graph, iters, pools):
    log("batch", capacity, graph, iters, pools)
    Rs, args, sc = _jobs(with_scenes=True)
    imgs, ms, res = ptmi.render_batch(Rs, args, pool_capacity=capacity, use_graph=graph, iters_per_graph=iters,
                                      pools=pools)
    torch.cuda.synchronize()
    _oracle_check(imgs, args, sc, f"batch capacity {capacity} pools {pools}")
    for j, (R, kw) in enumerate(zip(Rs, args)):
        ref = R.render(mode="wave", job=j, **kw).cpu().numpy()
        assert np.array_equal(imgs[j].cpu().numpy().view(np.uint32), ref.view(np.uint32)), j
    assert res["path_samples"] == sum(R.width * R.height * kw["spp"] for R, kw in zip(Rs, args))
    assert (ms > 0).all() and res["iterations"] > 0
    log("job ms", ms, res["iterations"], "iterations", res["launches"], "launches")


def test_batch_rejects_bad_options():
    Rs, args = _jobs()
    with pytest.raises(ptmi.PtError):
        ptmi.render_batch(Rs, args, iters_per_graph=3)
    with pytest.raises(ptmi.PtError):
        ptmi.render_batch(Rs, args, pool_capacity=8)
    with pytest.raises(ptmi.PtError):
        ptmi.render_batch(Rs, args, pools=5)  # more than four pools
    with pytest.raises(ptmi.PtError):
        ptmi.render_batch(Rs[:2], args[:2], pools=3)  # a pool without a job
    with pytest.raises(ptmi.PtError):
        ptmi.render_batch(Rs, args, pool_capacity=128, pools=4)  # 32 slots per pool


def test_batch_mixed_samplers_equal_standalone():
    log("batch mixed samplers")
    Rs, args, sc = _jobs(with_scenes=True)
    for j, a in enumerate(args):
        a["sampler"] = "halton" if j % 2 else "philox"
    imgs, ms, res = ptmi.render_batch(Rs, args, pool_capacity=500, use_graph=True, iters_per_graph=4)
    torch.cuda.synchronize()
    _oracle_check(imgs, args, sc, "batch mixed samplers")
    for j, (R, kw) in enumerate(zip(Rs, args)):
        ref = R.render(mode="wave", job=j, **kw).cpu().numpy()
        assert np.array_equal(imgs[j].cpu().numpy().view(np.uint32), ref.view(np.uint32)), j
