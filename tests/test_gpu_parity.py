"""Parity of the HIP path (through the C ABI) with the FP64 CPU oracle.

Bar: the weighted half grid is bit-identical (FP64 path: to the oracle's FP64 modes; FP32
path: to the oracle's modes rounded to FP32 factor by factor); fields and maps agree with
the FP64 oracle to max|gpu - oracle| / rms(oracle) <= 1e-5 (FP32) and <= 1e-12 (FP64).
"""
import numpy as np
import pytest

from oracle import field as ofield
from oracle import gather as ogather
from oracle import noise as onoise
from paper_2507_15703_amd import workloads

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = {"f32": 1e-5, "f64": 1e-12}
NPDT = {"f32": np.float32, "f64": np.float64}


@pytest.fixture(scope="module")
def cmbx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2507_15703_amd import cmbx as c
    c.lib()
    return c


def _plan(cmbx, N, L, dt, batch=1, interp="trilinear", table=None):
    p = cmbx.Plan(N, L, dt, batch=batch, interp=interp)
    k, pk = table if table is not None else workloads.powerlaw_cutoff_table(N, L, kc_modes=max(2, N // 4))
    p.spectrum_table(k, pk)
    return p, (k, pk)


def _rel(gpu, ref):
    ref = np.asarray(ref, dtype=np.float64)
    return np.max(np.abs(np.asarray(gpu, dtype=np.float64) - ref)) / np.sqrt(np.mean(ref**2))


def _bits(a):
    a = np.ascontiguousarray(a)
    return a.view(np.uint32 if a.dtype in (np.float32, np.complex64) else np.uint64)


# ------------------------------------------------------------------ noise (bit-exact)
@pytest.mark.parametrize("dt", ["f32", "f64"])
@pytest.mark.parametrize("N", [8, 12, 16, 24, 48, 64])
def test_noise_bit_exact(cmbx, N, dt):
    L = 1.0 + N / 100.0
    p, (k, pk) = _plan(cmbx, N, L, dt)
    for seed in (0, 1, (5 << 32) | 77, 2**64 - 1):
        gpu = p.debug_noise(seed).cpu().numpy()
        ref = onoise.halfgrid(N, L, seed, k, pk, dtype=NPDT[dt])
        assert np.array_equal(_bits(gpu), _bits(ref)), (N, dt, seed)
    p.close()


@pytest.mark.parametrize("dt", ["f32", "f64"])
@pytest.mark.parametrize("N", [16, 48, 64])
def test_noise_bit_exact_zero_weights(cmbx, N, dt):
    """A spectrum that ends at the box's isotropic band limit pi N / L (as the programme's
    solutions do): the modes beyond it have zero weight and are exactly +0, the rest are
    the oracle's bits."""
    L = 1.0
    k, pk = workloads.powerlaw_cutoff_table(N, L, kc_modes=N // 4)
    keep = k <= np.pi * N / L
    p, _ = _plan(cmbx, N, L, dt, table=(k[keep], pk[keep]))
    for seed in (3, 2**40 + 5):
        gpu = p.debug_noise(seed).cpu().numpy()
        ref = onoise.halfgrid(N, L, seed, k[keep], pk[keep], dtype=NPDT[dt])
        assert np.array_equal(_bits(gpu), _bits(ref)), (N, dt, seed)
        assert np.count_nonzero(_bits(ref)) < 0.75 * _bits(ref).size   # the corners are zero
    p.close()


def test_noise_bit_exact_256(cmbx):
    N, L = 256, 1.0
    p, (k, pk) = _plan(cmbx, N, L, "f32")
    gpu = p.debug_noise(1).cpu().numpy()
    ref = onoise.halfgrid(N, L, 1, k, pk, dtype=np.float32)
    assert np.array_equal(_bits(gpu), _bits(ref))
    p.close()


def test_largest_box_1024_sampled(cmbx):
    """The largest compiled box, 1024^3 FP32 (the precision-study size): the generic modes
    of sampled x-planes are bit-identical to the oracle's, and the FP32 map of a 40-degree
    cap agrees with the FP64 plan's to the FP32 bar (both plans are checked against the
    oracle at smaller sizes; the full 1024^3 oracle comparison is the precision study)."""
    from oracle import spectrum as ospec
    N, L, seed = 1024, 1.0, 11
    k, pk = workloads.powerlaw_cutoff_table(N, L, kc_modes=N // 4)
    p32, _ = _plan(cmbx, N, L, "f32", interp="tricubic", table=(k, pk))
    half, _ = ospec.weight_tables(N, L, k, pk)
    grid = p32.debug_noise(seed)
    for ix in (0, 1, 511, 512, 1023):
        g_re, g_im = onoise.unit_normals(N, seed, np.array([ix]), np.float32)
        w = half[ospec.mode_m(N, np.array([ix]))].astype(np.float32)
        ref = np.empty((N, N // 2 + 1), dtype=np.complex64)
        ref.real, ref.imag = (w * g_re)[0], (w * g_im)[0]
        got = grid[ix].cpu().numpy()
        # generic modes (the planes iz = 0 and N/2 follow the Hermitian rule, checked at smaller N)
        assert np.array_equal(_bits(got[:, 1:N // 2]), _bits(ref[:, 1:N // 2])), ix
    del grid
    dirs = torch.tensor(workloads.cap_directions(40.0, 1024, 1024), device="cuda")
    m32 = p32.simulate_patch(seed, 0.45, dirs).cpu().numpy()[0]
    p32.close()
    p64, _ = _plan(cmbx, N, L, "f64", interp="tricubic", table=(k, pk))
    m64 = p64.simulate_patch(seed, 0.45, dirs).cpu().numpy()[0]
    p64.close()
    assert np.all(np.isfinite(m32)) and _rel(m32, m64) <= 1e-5


# ------------------------------------------------------------------ field
@pytest.mark.parametrize("dt", ["f32", "f64"])
@pytest.mark.parametrize("N", [8, 12, 16, 24, 32, 48, 64, 96, 128])
def test_field_matches_oracle(cmbx, N, dt):
    L = 1.0
    p, (k, pk) = _plan(cmbx, N, L, dt)
    gpu = p.debug_field(7).cpu().numpy()
    ref = ofield.field(onoise.halfgrid(N, L, 7, k, pk, dtype=np.float64))
    assert _rel(gpu, ref) <= TOL[dt], (N, dt)
    p.close()


def _support_table(N, L, frac):
    """A power-law table that ends at frac x the band limit pi N / L: the modes beyond carry
    no power, so pass x skips their draws (and whole tiles) and pass y skips their lines."""
    k, pk = workloads.powerlaw_cutoff_table(N, L, kc_modes=max(2, N // 4))
    keep = k <= frac * np.pi * N / L
    return k[keep], pk[keep]


@pytest.mark.parametrize("dt", ["f32", "f64"])
@pytest.mark.parametrize("N", [8, 16, 48, 64, 128])
def test_field_limited_support_matches_oracle(cmbx, N, dt):
    L = 1.0
    table = _support_table(N, L, 0.55)
    p, _ = _plan(cmbx, N, L, dt, table=table)
    ref = ofield.field(onoise.halfgrid(N, L, 5, *table, dtype=np.float64))
    gpu = p.debug_field(5).cpu().numpy()
    assert _rel(gpu, ref) <= TOL[dt], (N, dt)
    for txy in (8, 4, 2):   # other tiles: other zero-tile boundaries
        try:
            p.set_tiles(txy, 0)
        except cmbx.CmbxError:
            continue
        assert _rel(p.debug_field(5).cpu().numpy(), ref) <= TOL[dt], (N, dt, txy)
    p.close()


@pytest.mark.parametrize("dt", ["f32", "f64"])
def test_support_shrinks_after_wide_run(cmbx, dt):
    """Parts of the workspace beyond the support are neither written nor read: a narrow
    spectrum after a full-band run on the same plan still matches the oracle."""
    N, L = 64, 1.0
    p, _ = _plan(cmbx, N, L, dt)
    f = torch.empty((N, N, N), dtype=p.torch_dtype, device="cuda")
    cmbx.debug_field(p.handle, 9, f.data_ptr())   # leaves a full-band field in f
    for frac in (0.3, 0.05):
        table = _support_table(N, L, frac)
        p.spectrum_table(*table)
        ref = ofield.field(onoise.halfgrid(N, L, 6, *table, dtype=np.float64))
        cmbx.debug_field(p.handle, 6, f.data_ptr())
        assert _rel(f.cpu().numpy(), ref) <= TOL[dt], (dt, frac)
    p.close()


def test_ensemble_rejects_grown_support(cmbx):
    """An ensemble's kernels skip what lay beyond each plan's support when it was created:
    a narrower spectrum later is fine, a wider one is refused until the ensemble is made
    again."""
    N = 48
    narrow, wide = _support_table(N, 1.0, 0.5), _support_table(N, 1.0, 1.0)
    p, _ = _plan(cmbx, N, 1.0, "f32", interp="tricubic", table=narrow)
    dirs = torch.tensor(workloads.cap_directions(25.0, 16, 64), device="cuda")
    out = torch.empty((1, dirs.shape[0]), dtype=torch.float32, device="cuda")
    for mode in ("chained", "pipelined"):
        p.spectrum_table(*narrow)
        ens = cmbx.Ensemble([dict(plan=p, seed=3, r=0.45, dirs=dirs, out=out)], mode=mode)
        p.spectrum_table(*_support_table(N, 1.0, 0.3))
        ens.launch()
        torch.cuda.synchronize()
        ref = p.simulate_patch(3, 0.45, dirs).cpu().numpy()[0]
        assert _rel(out.cpu().numpy()[0], ref) <= 1e-6, mode
        p.spectrum_table(*wide)
        with pytest.raises(cmbx.CmbxError) as e:
            ens.launch()
        assert e.value.code == cmbx.ESTATE
        ens.close()
    p.close()


def _turned(dirs, k):
    """The cap turned to another axis: a cyclic shift of the coordinates and, for odd k, a
    reflection (caps at -z, +x, -y, ...), so the stencils cross the periodic boundary
    along every axis when r is close to L/2."""
    d = np.roll(dirs, k // 2, axis=1)
    return -d if k % 2 else d


@pytest.mark.parametrize("interp", ["trilinear", "tricubic"])
@pytest.mark.parametrize("dt", ["f32", "f64"])
@pytest.mark.parametrize("N", [12, 48, 64, 128])
def test_pruned_maps_equal_whole_field_maps(cmbx, N, dt, interp):
    """Maps made from the part of the field the stencils read are bit-identical to maps of
    the whole field: every value the gather reads is made by the same arithmetic. Caps on
    all six half-axes near the box faces (r = 0.49 L) wrap the stencils; the pruning plan
    keeps whatever an earlier call left outside the new footprint."""
    L = 1.0
    k, pk = workloads.powerlaw_cutoff_table(N, L, kc_modes=max(2, N // 4))
    whole = cmbx.Plan(N, L, dt, batch=2, interp=interp, prune=False)
    pruned = cmbx.Plan(N, L, dt, batch=2, interp=interp)
    for p in (whole, pruned):
        p.spectrum_table(k, pk)
    base = workloads.cap_directions(20.0, 24, 96)
    for turn in range(6):
        for r in (0.49, 0.3):
            dirs = torch.tensor(_turned(base, turn), device="cuda")
            a = whole.simulate_patch(11 + turn, r, dirs).cpu().numpy()
            b = pruned.simulate_patch(11 + turn, r, dirs).cpu().numpy()
            assert np.array_equal(_bits(a), _bits(b)), (N, dt, interp, turn, r)
    whole.close()
    pruned.close()


def _footprint_ref(N, L, r, dirs, K):
    """What the K-point stencils read, from the definition: node i0 + a (mod N) on each
    axis, i0 = floor(p) mod N - (1 if K = 4), p = (r n + L/2) N / L in FP64 as the gather
    forms it (no fused multiply-add)."""
    p = (r * dirs + 0.5 * L) * (N / L)
    base = np.floor(p).astype(np.int64) % N - (1 if K == 4 else 0)
    nb = (N + 7) // 8
    planes = np.zeros(N, np.uint8)
    blocks = np.zeros((N, nb), np.uint8)
    zblocks = np.zeros((N + 31) // 32, np.uint8)
    for a in range(K):
        ix = (base[:, 0] + a) % N
        planes[ix] = 1
        zblocks[((base[:, 2] + a) % N) // 32] = 1
        for b in range(K):
            blocks[ix, ((base[:, 1] + b) % N) // 8] = 1
    return planes, blocks, zblocks


@pytest.mark.parametrize("interp", ["trilinear", "tricubic"])
@pytest.mark.parametrize("N", [12, 64, 512])
def test_footprint_matches_definition(cmbx, N, interp):
    """Marks (planes, row blocks, z blocks) bit-exact against the definition; the z list
    holds each block of `lines` lines with a marked line exactly once, the plane list each
    marked plane once."""
    L, K = 1.0, (4 if interp == "tricubic" else 2)
    p = cmbx.Plan(N, L, "f32", interp=interp)
    for turn, (theta, r) in enumerate([(20.0, 0.49), (35.0, 0.3), (5.0, 0.45)]):
        dn = _turned(workloads.cap_directions(theta, 48, 192), turn)
        planes, blocks, zblocks, lines, lst, plist = p.debug_footprint(r, torch.tensor(dn, device="cuda"))
        rp, rb, rz = _footprint_ref(N, L, r, dn, K)
        assert np.array_equal(planes, rp) and np.array_equal(blocks, rb), (N, interp, turn)
        assert np.array_equal(zblocks, rz), (N, interp, turn)
        assert lines in cmbx.tile_choices("f32", N, 1)
        line_marked = rb[np.arange(N * N) // N, (np.arange(N * N) % N) // 8].astype(bool)
        want = np.nonzero(line_marked.reshape(-1, lines).any(axis=1))[0]
        assert np.array_equal(lst, want.astype(np.uint32)), (N, interp, turn)
        assert np.array_equal(plist, np.nonzero(rp)[0].astype(np.uint32)), (N, interp, turn)
    p.close()


@pytest.mark.parametrize("mode", ["chained", "pipelined"])
def test_pruned_ensemble_matches_whole_field(cmbx, mode):
    """Ensembles of pruning plans (footprints made inside the graph at every launch) against
    whole-field maps; new directions between launches are picked up."""
    jobs, whole = [], []
    for i, (N, theta) in enumerate([(48, 12.0), (48, 35.0), (64, 25.0), (64, 8.0)]):
        k, pk = workloads.powerlaw_cutoff_table(N, 1.0, kc_modes=N // 4)
        p = cmbx.Plan(N, 1.0, "f32", interp="tricubic")
        p.spectrum_table(k, pk)
        w = cmbx.Plan(N, 1.0, "f32", interp="tricubic", prune=False)
        w.spectrum_table(k, pk)
        dirs = torch.tensor(_turned(workloads.cap_directions(theta, 16, 64), i), device="cuda")
        out = torch.empty((1, dirs.shape[0]), dtype=torch.float32, device="cuda")
        jobs.append(dict(plan=p, seed=40 + i, r=0.45, dirs=dirs, out=out))
        whole.append(w)
    ens = cmbx.Ensemble([dict(j) for j in jobs], mode=mode)
    for launch in range(2):
        if launch:
            for i, j in enumerate(jobs):   # same buffers, other directions
                j["dirs"].copy_(torch.tensor(_turned(workloads.cap_directions(20.0, 16, 64), i + 3), device="cuda"))
        ens.launch()
        torch.cuda.synchronize()
        for j, w in zip(jobs, whole):
            ref = w.simulate_patch(j["seed"], j["r"], j["dirs"]).cpu().numpy()[0]
            assert _rel(j["out"].cpu().numpy()[0], ref) <= 1e-6, (mode, launch, j["plan"].N)
    ens.close()
    for j, w in zip(jobs, whole):
        j["plan"].close()
        w.close()


def test_pipelined_ensemble_limited_support(cmbx):
    """The fused pipeline takes each item's support bound from its own weight table."""
    jobs = []
    for i, (N, frac) in enumerate([(48, 0.4), (48, 1.0), (48, 0.7), (64, 0.5), (64, 0.9)]):
        table = _support_table(N, 1.0, frac)
        p, _ = _plan(cmbx, N, 1.0, "f32", interp="tricubic", table=table)
        dirs = torch.tensor(workloads.cap_directions(25.0, 16, 64), device="cuda")
        out = torch.empty((1, dirs.shape[0]), dtype=torch.float32, device="cuda")
        jobs.append(dict(plan=p, seed=70 + i, r=0.45, dirs=dirs, out=out))
    ens = cmbx.Ensemble([dict(j) for j in jobs], mode="pipelined")
    ens.launch()
    torch.cuda.synchronize()
    for j in jobs:
        ref = j["plan"].simulate_patch(j["seed"], j["r"], j["dirs"]).cpu().numpy()[0]
        assert _rel(j["out"].cpu().numpy()[0], ref) <= 1e-6, j["plan"].N
    ens.close()
    for j in jobs:
        j["plan"].close()


@pytest.mark.parametrize("dt", ["f32", "f64"])
@pytest.mark.parametrize("N", [64, 384])
def test_field_alt_tiles_agree(cmbx, N, dt):
    """Every compiled tile shape gives the same field up to rounding (the compiler may
    contract multiply-adds differently per instantiation). Bar for FP32: the three passes'
    rounding gives each point a relative spread of about eps sqrt(3 log2 N) (3e-7 at
    N = 384, eps = 6e-8), whose maximum over N^3 points is about 5.5 sigma = 1.6e-6: 2e-6.
    FP64: the same reasoning at eps = 1.1e-16, 1e-14."""
    p, (k, pk) = _plan(cmbx, N, 1.0, dt)
    base = p.debug_field(3).cpu().numpy()
    if N <= 64:
        ref = ofield.field(onoise.halfgrid(N, 1.0, 3, k, pk))
        assert _rel(base, ref) <= TOL[dt]
    tried = 0
    for txy, lz in [(16, 0), (8, 0), (4, 0), (2, 0), (0, 32), (0, 16), (0, 8), (0, 4), (0, 2)]:
        try:
            p.set_tiles(txy, lz)
        except cmbx.CmbxError:
            continue
        tried += 1
        err = _rel(p.debug_field(3).cpu().numpy(), base)
        assert err <= (2e-6 if dt == "f32" else 1e-14), (txy, lz, err)
    assert tried >= 2
    p.close()


@pytest.mark.parametrize("dt", ["f32", "f64"])
def test_autotune_picks_compiled_shapes(cmbx, dt, tmp_path):
    """The chain-timed autotuner returns compiled shapes, sets them on the plan (the field
    still matches the oracle) and caches them."""
    N = 48
    p, (k, pk) = _plan(cmbx, N, 1.0, dt)
    cache = str(tmp_path / "tune.json")
    t = p.autotune(reps=2, cache_path=cache)
    assert not t["cached"]
    assert t["tile_x"] in cmbx.tile_choices(dt, N, 0) and t["tile_y"] in cmbx.tile_choices(dt, N, 0)
    assert t["lines_z"] in cmbx.tile_choices(dt, N, 1)
    assert all(m > 0 for m in t["ms"])
    ref = ofield.field(onoise.halfgrid(N, 1.0, 4, k, pk))
    assert _rel(p.debug_field(4).cpu().numpy(), ref) <= TOL[dt]
    again = p.autotune(reps=2, cache_path=cache)
    assert again["cached"] and again["tile_x"] == t["tile_x"] and again["lines_z"] == t["lines_z"]
    p.close()


def test_autotune_on_a_maps_pixels(cmbx):
    """Tuning on a map's pixels (pruned chains) returns compiled shapes, caches nothing,
    and the map afterwards still equals the whole-field map."""
    N = 64
    k, pk = workloads.powerlaw_cutoff_table(N, 1.0, kc_modes=N // 4)
    p = cmbx.Plan(N, 1.0, "f32", interp="tricubic")
    w = cmbx.Plan(N, 1.0, "f32", interp="tricubic", prune=False)
    for q in (p, w):
        q.spectrum_table(k, pk)
    dirs = torch.tensor(workloads.cap_directions(20.0, 32, 128), device="cuda")
    t = p.autotune(reps=2, r=0.45, dirs=dirs)
    assert not t["cached"] and t["tile_x"] in cmbx.tile_choices("f32", N, 0)
    assert t["lines_z"] in cmbx.tile_choices("f32", N, 1) and all(m > 0 for m in t["ms"])
    # the same stage plans too: a plan 1 transform rounds differently from plan 0
    w.set_tiles(0, t["lines_z"], tile_x=t["tile_x"], tile_y=t["tile_y"], plans=t["plans"])
    a = p.simulate_patch(8, 0.45, dirs).cpu().numpy()
    b = w.simulate_patch(8, 0.45, dirs).cpu().numpy()
    assert np.array_equal(_bits(a), _bits(b))
    p.close()
    w.close()


@pytest.mark.parametrize("dt", ["f32", "f64"])
def test_field_256(cmbx, dt):
    N, L = 256, 1.0
    p, (k, pk) = _plan(cmbx, N, L, dt)
    gpu = p.debug_field(1).cpu().numpy()
    ref = ofield.field(onoise.halfgrid(N, L, 1, k, pk, dtype=np.float64), workers=-1)
    assert _rel(gpu, ref) <= TOL[dt]
    p.close()


# ------------------------------------------------------------------ gather
@pytest.mark.parametrize("dt", ["f32", "f64"])
@pytest.mark.parametrize("interp", ["trilinear", "tricubic"])
def test_gather_matches_oracle(cmbx, dt, interp):
    N, L = 32, 2.0
    p, _ = _plan(cmbx, N, L, dt, interp=interp)
    rng = np.random.default_rng(9)
    fld = rng.standard_normal((N, N, N))
    ft = torch.tensor(fld.astype(NPDT[dt]), device="cuda")
    cases = [
        (0.7, workloads.random_directions(1000, 1)),
        (0.9999, workloads.random_directions(257, 2)),          # stencils wrap at the edge
        (0.25, np.array([[0, 0, 1.0], [1, 0, 0], [0, -1, 0]])),  # exactly on nodes: 0.25 * 32 / 2 = 4
        (0.5, workloads.random_directions(1, 3)),                 # a single pixel
    ]
    for r, dirs in cases:
        d = torch.tensor(dirs, device="cuda")
        gpu = p.debug_gather(ft, r, d).cpu().numpy()
        ref = ogather.gather(fld.astype(NPDT[dt]).astype(np.float64), L, r, dirs, interp)
        assert _rel(gpu, ref) <= (2e-6 if dt == "f32" else 1e-13), (r, interp, dt)
    p.close()


# ------------------------------------------------------------------ end to end
def test_simulate_config_small_fp64(cmbx):
    """64^3 FP64, r = 0.4 L, cap 20 deg (128 x 512 pixels), trilinear, seed 0."""
    N, L, r = 64, 1.0, 0.4
    table = workloads.powerlaw_cutoff_table(N, L, kc_modes=16)
    p, (k, pk) = _plan(cmbx, N, L, "f64", interp="trilinear", table=table)
    dirs = workloads.cap_directions(20.0, 128, 512)
    out = p.simulate_patch(0, r, torch.tensor(dirs, device="cuda")).cpu().numpy()
    h = onoise.halfgrid(N, L, 0, k, pk)
    ref = ogather.gather(ofield.field(h), L, r, dirs, "trilinear")
    assert _rel(out[0], ref) <= 1e-12
    p.close()


@pytest.mark.parametrize("dt", ["f32", "f64"])
def test_simulate_batch_seeds(cmbx, dt):
    """Realisation b of a batch uses seed + b; every realisation matches the oracle."""
    N, L, r = 48, 1.0, 0.45
    p, (k, pk) = _plan(cmbx, N, L, dt, batch=3, interp="tricubic")
    dirs = workloads.cap_directions(35.0, 40, 77)
    out = p.simulate_patch(100, r, torch.tensor(dirs, device="cuda")).cpu().numpy()
    for b in range(3):
        ref = ogather.gather(ofield.field(onoise.halfgrid(N, L, 100 + b, k, pk)), L, r, dirs, "tricubic")
        assert _rel(out[b], ref) <= TOL[dt], b
    p.close()


def test_simulate_256_tricubic_fp32(cmbx):
    """256^3 FP32, r = 0.45 L, cap 30 deg as 1024 x 1024 pixels, tricubic, seed 1."""
    N, L, r = 256, 1.0, 0.45
    p, (k, pk) = _plan(cmbx, N, L, "f32", interp="tricubic")
    dirs = workloads.cap_directions(30.0, 1024, 1024)
    out = p.simulate_patch(1, r, torch.tensor(dirs, device="cuda")).cpu().numpy()
    fld = ofield.field(onoise.halfgrid(N, L, 1, k, pk), workers=-1)
    ref = ogather.gather(fld, L, r, dirs, "tricubic")
    assert _rel(out[0], ref) <= 1e-5
    p.close()


def test_errors_on_device(cmbx):
    p = cmbx.Plan(16, 1.0, "f32")
    d = torch.zeros((4, 3), dtype=torch.float64, device="cuda")
    d[:, 2] = 1
    with pytest.raises(cmbx.CmbxError) as e:
        p.simulate_patch(0, 0.3, d)
    assert e.value.code == cmbx.ESTATE
    k, pk = workloads.powerlaw_cutoff_table(16, 1.0)
    p.spectrum_table(k, pk)
    for bad_r in (0.0, -0.1, 0.5, 0.7):
        with pytest.raises(cmbx.CmbxError) as e:
            p.simulate_patch(0, bad_r, d)
        assert e.value.code == cmbx.EINVAL
    with pytest.raises(cmbx.CmbxError) as e:
        p.spectrum_table(k[::-1].copy(), pk)
    assert e.value.code == cmbx.EINVAL
    with pytest.raises(cmbx.CmbxError):
        p.set_tiles(5, 0)
    p.close()


def test_fault_injection_leaves_library_usable(cmbx, monkeypatch):
    """Failures forced from the host (CMBX_FAULT) return their codes and leave nothing
    behind: the next plan, ensemble and launch work and give the plain path's maps."""
    monkeypatch.setenv("CMBX_FAULT", "alloc")
    with pytest.raises(cmbx.CmbxError) as e:
        cmbx.Plan(32, 1.0, "f32")
    assert e.value.code == cmbx.ENOMEM
    monkeypatch.delenv("CMBX_FAULT")
    p, _ = _plan(cmbx, 32, 1.0, "f32", interp="tricubic")
    dirs = torch.tensor(workloads.cap_directions(20.0, 16, 64), device="cuda")
    out = torch.empty((1, dirs.shape[0]), dtype=torch.float32, device="cuda")
    job = dict(plan=p, seed=9, r=0.45, dirs=dirs, out=out)
    monkeypatch.setenv("CMBX_FAULT", "capture")
    with pytest.raises(cmbx.CmbxError) as e:
        cmbx.Ensemble([job], mode="chained")
    assert e.value.code == cmbx.EHIP
    monkeypatch.delenv("CMBX_FAULT")
    ens = cmbx.Ensemble([job], mode="chained")
    monkeypatch.setenv("CMBX_FAULT", "launch")
    with pytest.raises(cmbx.CmbxError) as e:
        ens.launch()
    assert e.value.code == cmbx.EHIP
    monkeypatch.delenv("CMBX_FAULT")
    out.fill_(float("nan"))
    ens.launch()
    torch.cuda.synchronize()
    ref = p.simulate_patch(9, 0.45, dirs).cpu().numpy()
    assert _rel(out.cpu().numpy()[0], ref[0]) <= 1e-6
    ens.close()
    p.close()


# ------------------------------------------------------------------ ensemble (graph)
@pytest.mark.parametrize("mode", ["chained", "pipelined", "auto", "chained-2-lanes", "chained-4-lanes"])
@pytest.mark.parametrize("dt", ["f32", "f64"])
def test_ensemble_graph_matches_plain_and_oracle(cmbx, dt, mode):
    """The hipGraph ensemble (mixed sizes, batches, both interpolants; one lane or several) gives
    the plain path's maps up to rounding, and the oracle's to the parity bar, on every
    replay."""
    specs = [(32, 3, 12.0, "tricubic"), (48, 2, 25.0, "trilinear"), (32, 1, 33.0, "tricubic"),
             (64, 2, 18.0, "tricubic"), (48, 1, 40.0, "tricubic")]
    jobs, plans = [], []
    for i, (N, batch, th, interp) in enumerate(specs):
        p, (k, pk) = _plan(cmbx, N, 1.0, dt, batch=batch, interp=interp)
        plans.append((p, k, pk))
        dirs_np = workloads.cap_directions(th, 20, 64 + 7 * i)
        dirs = torch.tensor(dirs_np, device="cuda")
        out = torch.empty((batch, dirs.shape[0]), dtype=p.torch_dtype, device="cuda")
        jobs.append(dict(plan=p, seed=50 + 10 * i, r=0.45, dirs=dirs, out=out, dirs_np=dirs_np, k=k, pk=pk))
    lanes = int(mode.split("-")[1]) if mode.endswith("lanes") else None
    mode = mode.split("-")[0]
    ens = cmbx.Ensemble([{kk: j[kk] for kk in ("plan", "seed", "r", "dirs", "out")} for j in jobs], mode=mode,
                        lanes=lanes)
    assert len(ens.modes) == 3 and (mode == "auto" or set(ens.modes) == {mode})
    assert ens.lanes == (lanes if lanes else ens.lanes) and 1 <= ens.lanes <= 4
    if mode == "pipelined":
        assert ens.lanes == 1
    refs = []
    for j in jobs:
        ref = j["plan"].simulate_patch(j["seed"], j["r"], j["dirs"]).cpu().numpy()
        refs.append(ref)
    for rep in range(3):
        for j in jobs:
            j["out"].fill_(float("nan"))
        ens.launch()
        torch.cuda.synchronize()
        for j, ref in zip(jobs, refs):
            got = j["out"].cpu().numpy()
            for b in range(got.shape[0]):
                assert _rel(got[b], ref[b]) <= (1e-6 if dt == "f32" else 1e-14), (rep, j["plan"].N, b)
    # against the oracle, once per job and realisation
    for j in jobs:
        p = j["plan"]
        got = j["out"].cpu().numpy()
        for b in range(p.batch):
            fld = ofield.field(onoise.halfgrid(p.N, 1.0, j["seed"] + b, j["k"], j["pk"]))
            ref = ogather.gather(fld, 1.0, j["r"], j["dirs_np"], "tricubic" if p.interp == cmbx.TRICUBIC else "trilinear")
            assert _rel(got[b], ref) <= TOL[dt]
    ens.close()
    for p, _, _ in plans:
        p.close()


def test_ensemble_512_sampled(cmbx):
    """The bench's launch configuration at full size: four 512^3 FP32 boxes pipelined in one
    graph. Pixels sampled from each map are checked against the plain path, and the maps'
    variance against the lattice prediction sum P_box (a property at any size)."""
    from oracle import spectrum as ospec
    jobs_meta = [j for j in workloads.ensemble_jobs() if j["N"] == 512]
    jobs = []
    for j in jobs_meta:
        p = cmbx.Plan(512, 1.0, "f32", interp="tricubic")
        k, pk = workloads.powerlaw_cutoff_table(512, 1.0, kc_modes=128)
        p.spectrum_table(k, pk * j["amp"])
        dirs = torch.tensor(workloads.cap_directions(j["theta_deg"], j["n_ring"], j["n_phi"]), device="cuda")
        out = torch.empty((1, dirs.shape[0]), dtype=torch.float32, device="cuda")
        jobs.append(dict(plan=p, seed=j["seed"], r=0.45, dirs=dirs, out=out, amp=j["amp"], k=k, pk=pk))
    ens = cmbx.Ensemble([{kk: j[kk] for kk in ("plan", "seed", "r", "dirs", "out")} for j in jobs],
                        mode="pipelined")
    ens.launch()
    torch.cuda.synchronize()
    for j in jobs:
        got = j["out"].cpu().numpy()[0]
        ref = j["plan"].simulate_patch(j["seed"], j["r"], j["dirs"]).cpu().numpy()[0]
        idx = np.random.default_rng(j["seed"]).choice(got.size, 4096, replace=False)
        assert _rel(got[idx], ref[idx]) <= 1e-6
        assert np.all(np.isfinite(got))
        # <T^2> over a cap of >= 4e5 correlated pixels is a noisy estimate of xi(0); check
        # it is within a generous factor of the lattice variance
        xi0 = ospec.lattice_xi0(512, 1.0, j["k"], j["pk"])
        assert 0.5 < np.mean(got.astype(np.float64) ** 2) / xi0 < 2.0
    ens.close()
    for j in jobs:
        j["plan"].close()


def test_ensemble_mixed_sizes_full_workload(cmbx):
    """The mixed-size ensemble workload (16 x 128^3 + 8 x 256^3 + 4 x 384^3 + 4 x 512^3 FP32,
    caps of 10-40 degrees, tricubic) in one auto-mode ensemble gives every job's plain-path
    map (sampled pixels, to rounding) on two replays."""
    jobs = []
    for j in workloads.ensemble_jobs():
        N = j["N"]
        k, pk = workloads.powerlaw_cutoff_table(N, 1.0, kc_modes=N // 4)
        p, _ = _plan(cmbx, N, 1.0, "f32", interp="tricubic", table=(k, pk * j["amp"]))
        dirs = torch.tensor(workloads.cap_directions(j["theta_deg"], j["n_ring"], j["n_phi"]), device="cuda")
        out = torch.empty((1, dirs.shape[0]), dtype=torch.float32, device="cuda")
        jobs.append(dict(plan=p, seed=j["seed"], r=0.45, dirs=dirs, out=out))
    ens = cmbx.Ensemble([dict(j) for j in jobs], mode="auto")
    assert len(ens.modes) == 4
    refs = [j["plan"].simulate_patch(j["seed"], j["r"], j["dirs"]).cpu().numpy()[0] for j in jobs]
    for rep in range(2):
        for j in jobs:
            j["out"].fill_(float("nan"))
        ens.launch()
        torch.cuda.synchronize()
        for i, (j, ref) in enumerate(zip(jobs, refs)):
            got = j["out"].cpu().numpy()[0]
            idx = np.random.default_rng(i).choice(got.size, min(got.size, 8192), replace=False)
            assert np.all(np.isfinite(got)) and _rel(got[idx], ref[idx]) <= 1e-6, (rep, i, j["plan"].N)
    ens.close()
    for j in jobs:
        j["plan"].close()
