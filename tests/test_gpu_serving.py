"""Serving on the GPU: requests of uneven resolution and level selection served concurrently
(4 slots, Poisson arrivals) give the same images as each request rendered alone, their device
intervals (events on the slot streams) overlap, and what the device reserves for the process
never passes the budget."""
import numpy as np
import pytest

from paper_2408_12894_amd import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

RES = ((320, 180), (640, 360), (256, 256), (480, 270))


@pytest.fixture(scope="module")
def stack():
    from paper_2408_12894_amd import render
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    sizes = (20_000, 50_000, 100_000, 150_000, 200_000)
    return [render.GaussianLevel.from_scene(s) for s in synth.level_stack(sizes=sizes)]


def alone(stack, trace):
    from paper_2408_12894_amd import render
    r = render.Renderer(0)
    out = {}
    for q in trace:
        if q.l_start == q.l_end:
            img = r.render_level(stack[q.l_start - 1], q.camera)[0]
        else:
            img = r.render_selective(stack, q.l_start, q.l_end, synth.LEVEL_BANDS, q.camera.campos, q.camera)[0]
        out[q.rid] = img.cpu().numpy()
    r.close()
    return out


def test_mix_equals_alone(stack):
    from paper_2408_12894_amd import serving
    print("[case] 32 requests, 4 slots, generous budget", flush=True)
    trace = synth.serving_trace(seed=31, count=32, mean_gap_s=0.001, resolutions=RES)
    ref = alone(stack, trace)
    recs, st = serving.serve_trace(stack, trace, n_slots=4, budget_bytes=8 << 30, keep_images=True)
    print(st, flush=True)
    assert st["completed"] == 32 and st["rejected"] == 0
    assert st["peak_bytes"] <= st["budget_bytes"] and st["device_peak_reserved_bytes"] <= st["budget_bytes"]
    # requests ran on the device at the same time: their event intervals intersect
    assert st["device_overlapping"] >= 2 and st["device_max_in_flight"] >= 2
    assert all(r.dev_end_ms > r.dev_start_ms for r in recs)
    for rec in recs:
        np.testing.assert_array_equal(rec.result["image"].cpu().numpy(), ref[rec.rid])


def test_saturated_slots_overlap_on_the_device(stack):
    """All requests arrive at once: with 4 slots the device runs several of them at a time."""
    from paper_2408_12894_amd import serving
    print("[case] 48 requests at once, 4 slots", flush=True)
    trace = synth.serving_trace(seed=34, count=48, mean_gap_s=0.001, resolutions=RES)
    recs, st = serving.serve_trace(stack, trace, n_slots=4, budget_bytes=8 << 30, time_scale=0.0)
    print(st, flush=True)
    assert st["completed"] == 48
    assert st["device_max_in_flight"] >= 3 and st["device_concurrency"] > 1.2


def test_tight_budget(stack):
    from paper_2408_12894_amd import serving
    print("[case] tight budget: defer and reject", flush=True)
    trace = synth.serving_trace(seed=32, count=24, mean_gap_s=0.0005, resolutions=RES)
    ref = alone(stack, trace)
    # the budget: what the device holds for the idle server (the stack, as torch reserved it)
    # plus 256 MiB, charged for every allocation at the most torch may newly reserve for it (a
    # 20 MiB segment for one of 1 to 10 MiB), so the smaller requests fit and the larger ones
    # are deferred or rejected
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    budget = torch.cuda.memory_reserved() + (256 << 20)
    recs, st = serving.serve_trace(stack, trace, n_slots=4, budget_bytes=budget, keep_images=True)
    print(st, flush=True)
    assert st["peak_bytes"] <= budget and st["device_peak_reserved_bytes"] <= budget
    assert st["deferrals"] + st["rejected"] > 0
    assert all(r.status in ("ok", "rejected") for r in recs)
    assert st["completed"] >= 1
    for rec in recs:
        if rec.status == "ok":
            np.testing.assert_array_equal(rec.result["image"].cpu().numpy(), ref[rec.rid])
    print(st)
