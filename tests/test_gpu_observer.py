"""Observer placed off the box centre (Sec. II D 1 centres the box on the cap's axis at
(1 + z_min)/2 of the radius, so the observer sits below the centre).

The HIP path against the oracle's gather with the same observer, on a HEALPix cap; maps
made from the footprint bit-identical to whole-field maps with the observer moved; and an
ensemble keeping the position its plan had at creation.
"""
import math

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2507_15703_amd import cmbx
    return cmbx, torch


def _rel(a, b):
    return float(np.max(np.abs(np.asarray(a, dtype=np.float64) - b)) / np.sqrt(np.mean(np.asarray(b) ** 2)))


@pytest.mark.parametrize("dtype,tol", [("f64", 1e-12), ("f32", 1e-5)])
@pytest.mark.parametrize("interp", ["trilinear", "tricubic"])
def test_offset_observer_matches_oracle(env, dtype, tol, interp):
    cmbx, torch = env
    from oracle import field as ofield
    from oracle import gather as ogather
    from oracle import healpix as hp
    from oracle import noise as onoise
    from paper_2507_15703_amd import workloads
    N, L, seed = 32, 1.0, 21
    theta = 30.0
    z_min = math.cos(math.radians(theta))
    # the cap's extent, 2 r sin(theta) across, fills most of the box once it is centred
    r = 0.8 * L / (2.0 * math.sin(math.radians(theta)))
    print(f"[observer] {dtype} {interp} N={N} r={r:.3f}", flush=True)
    k, p = workloads.powerlaw_cutoff_table(N, L, kc_modes=8)
    plan = cmbx.Plan(N, L, dtype, batch=1, interp=interp)
    plan.spectrum_table(k, p)
    obs = plan.observer_for_cap(r, z_min)
    plan.set_observer(obs)
    dirs = cmbx.healpix_cap(32, z_min)
    got = plan.simulate_patch(seed, r, dirs)
    torch.cuda.synchronize()
    fld = ofield.field(onoise.halfgrid(N, L, seed, k, p))
    ref = ogather.gather(fld, L, r, hp.cap_directions(32, z_min), interp, observer=obs)
    assert _rel(got.cpu().numpy()[0], ref) <= tol
    # the default observer would sample other cells
    far = ogather.gather(fld, L, r, hp.cap_directions(32, z_min), interp)
    assert _rel(far, ref) > 0.1
    plan.close()


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_pruned_maps_equal_whole_field_with_offset_observer(env, dtype):
    cmbx, torch = env
    from paper_2507_15703_amd import workloads
    N, L = 64, 1.0
    k, p = workloads.powerlaw_cutoff_table(N, L, kc_modes=16)
    z_min = math.cos(math.radians(20.0))
    r = 0.9
    obs = (0.5, 0.5, 0.5 - r * (1.0 + z_min) / 2.0)
    dirs = cmbx.healpix_cap(64, z_min)
    maps = []
    for prune in (True, False):
        plan = cmbx.Plan(N, L, dtype, batch=2, interp="tricubic", prune=prune)
        plan.spectrum_table(k, p)
        plan.set_observer(obs)
        maps.append(plan.simulate_patch(5, r, dirs).cpu().numpy())
        plan.close()
    np.testing.assert_array_equal(maps[0], maps[1])


def test_ensemble_keeps_observer_of_creation(env):
    cmbx, torch = env
    from paper_2507_15703_amd import workloads
    N, L, r = 48, 1.0, 0.8
    k, p = workloads.powerlaw_cutoff_table(N, L, kc_modes=12)
    z_min = math.cos(math.radians(25.0))
    obs = (0.5, 0.5, 0.5 - r * (1.0 + z_min) / 2.0)
    dirs = cmbx.healpix_cap(16, z_min)
    plan = cmbx.Plan(N, L, "f32", interp="tricubic")
    plan.spectrum_table(k, p)
    plan.set_observer(obs)
    out = torch.empty((1, dirs.shape[0]), dtype=torch.float32, device="cuda")
    ens = cmbx.Ensemble([dict(plan=plan, seed=9, r=r, dirs=dirs, out=out)], mode="chained")
    ref = plan.simulate_patch(9, r, dirs).cpu().numpy()[0]
    plan.set_observer((0.5, 0.5, 0.5))   # later changes do not reach the captured graph
    ens.launch()
    torch.cuda.synchronize()
    np.testing.assert_array_equal(out.cpu().numpy()[0], ref)
    ens.close()
    plan.close()


@pytest.mark.parametrize("mode", ["pipelined", "chained"])
def test_ensemble_modes_follow_moved_observer(env, mode):
    # the pipelined kernel carries the observer in its own arguments: both modes against
    # the plan's plain maps, for two plans with different observers
    cmbx, torch = env
    from paper_2507_15703_amd import workloads
    jobs, refs = [], []
    for i, (N, theta) in enumerate([(48, 20.0), (48, 30.0), (48, 12.0), (48, 25.0)]):
        k, p = workloads.powerlaw_cutoff_table(N, 1.0, kc_modes=12)
        z_min = math.cos(math.radians(theta))
        r = 0.7
        plan = cmbx.Plan(N, 1.0, "f32", interp="tricubic" if i % 2 == 0 else "trilinear")
        plan.spectrum_table(k, p)
        plan.set_observer(plan.observer_for_cap(r, z_min))
        dirs = cmbx.healpix_cap(16, z_min)
        out = torch.empty((1, dirs.shape[0]), dtype=torch.float32, device="cuda")
        jobs.append(dict(plan=plan, seed=70 + i, r=r, dirs=dirs, out=out))
        refs.append(plan.simulate_patch(70 + i, r, dirs).cpu().numpy()[0])
    print(f"[observer] ensemble {mode}", flush=True)
    ens = cmbx.Ensemble([dict(j) for j in jobs], mode=mode)
    for _ in range(2):
        ens.launch()
        torch.cuda.synchronize()
        for j, ref in zip(jobs, refs):
            got = j["out"].cpu().numpy()[0]
            assert np.max(np.abs(got - ref)) / np.sqrt(np.mean(ref**2)) <= 1e-6, (mode, j["plan"].N)
    ens.close()
    for j in jobs:
        j["plan"].close()


def test_cap_observer_centres_the_cap(env):
    """cmbx_plan_cap_observer / cmbx_slab_cap_observer (Sec. II D 1-2): with that observer the
    cap's z range, o_z + r [z_min, 1], is centred on the box's centre (cubic box) or on the
    middle of the slab's layers, and its axis runs through the centre in x and y."""
    cmbx, torch = env
    plan = cmbx.Plan(32, 2.0, "f32")
    for r, z_min in ((0.7, math.cos(math.radians(20.0))), (0.9, 0.0), (0.5, -0.5)):
        o = plan.observer_for_cap(r, z_min)
        assert o[0] == 1.0 and o[1] == 1.0
        assert (o[2] + r * z_min + o[2] + r) / 2 == pytest.approx(1.0, abs=1e-15)
    for bad in ((0.0, 0.5), (1.0, 1.5), (float("nan"), 0.5)):
        with pytest.raises(cmbx.CmbxError):
            plan.observer_for_cap(*bad)
    plan.close()
    s = cmbx.Slab("hybrid", 32, 16, 0.01, h=6, dtype="f32")
    o = s.observer_for_cap(0.2, 0.9)
    assert o[0] == o[1] == pytest.approx(0.16, abs=1e-15)
    assert (2 * o[2] + 0.2 * 0.9 + 0.2) / 2 == pytest.approx(2.5 * 0.01, abs=1e-15)   # middle of layers 0 .. 5
    with pytest.raises(cmbx.CmbxError):
        s.observer_for_cap(-1.0, 0.5)
    s.close()
