"""Python binding of the C ABI in ``include/cmbx.h`` (ctypes; argument marshalling only).

Every call goes to ``_lib/libcmbx.so``; all computation happens in its HIP kernels. Device
buffers are passed as torch CUDA tensors (or raw integer addresses); torch supplies device
memory and streams only. If the library is missing, loading raises: there is no fallback.

The function names follow the C ABI without the ``cmbx_`` prefix; ``Plan`` and
``Ensemble`` are small owners that release their handles.
"""
import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "_lib", "libcmbx.so")

OK, EINVAL, EUNSUPPORTED, ENOMEM, EHIP, ESTATE = 0, -1, -2, -3, -4, -5
F32, F64 = 1, 2
TRILINEAR, TRICUBIC = 1, 2
ENS_AUTO, ENS_CHAINED, ENS_PIPELINED = 0, 1, 2
SLAB_FLAT, SLAB_HYBRID = 1, 2
ENS_ONE_LANE, ENS_TWO_LANES, ENS_MAX_LANES = 0x100, 0x200, 4
OPT_INTERP, OPT_STREAM, OPT_TILE_XY, OPT_LINES_Z, OPT_TILE_X, OPT_TILE_Y, OPT_PRUNE, OPT_FIXED_DIRS = 1, 2, 3, 4, 5, 6, 7, 8
OPT_PLAN_X, OPT_PLAN_Y, OPT_PLAN_Z = 9, 10, 11
SLAB_OPT_DIRECT = 12
_DIRECT = {"auto": 0, "never": 1, "always": 2}

_DTYPES = {"f32": F32, "float32": F32, F32: F32, "f64": F64, "float64": F64, F64: F64}
_INTERPS = {"trilinear": TRILINEAR, "tricubic": TRICUBIC, TRILINEAR: TRILINEAR, TRICUBIC: TRICUBIC}

_lib = None


class CmbxError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"cmbx error {code}: {msg}")
        self.code = code


class _Job(ctypes.Structure):
    _fields_ = [("plan", ctypes.c_void_p), ("seed", ctypes.c_uint64), ("r", ctypes.c_double),
                ("dirs", ctypes.c_void_p), ("n_pix", ctypes.c_int64), ("out", ctypes.c_void_p)]


def lib():
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"HIP library not built: {LIB_PATH} (run paper_2507_15703_amd.build)")
        L = ctypes.CDLL(LIB_PATH)
        P, I, D, U64, I64 = ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_uint64, ctypes.c_int64
        sig = {
            "cmbx_plan_box": (I, [I, D, I, I, ctypes.POINTER(P)]),
            "cmbx_plan_destroy": (I, [P]),
            "cmbx_plan_set": (I, [P, I, I64]),
            "cmbx_plan_get": (I, [P, I, ctypes.POINTER(I64)]),
            "cmbx_plan_observer": (I, [P, D, D, D]),
            "cmbx_plan_cap_observer": (I, [P, D, D, ctypes.POINTER(D)]),
            "cmbx_plan_info": (I, [P, ctypes.POINTER(I), ctypes.POINTER(D), ctypes.POINTER(I), ctypes.POINTER(I),
                                   ctypes.POINTER(P)]),
            "cmbx_spectrum_table": (I, [P, P, P, I64]),
            "cmbx_simulate_patch": (I, [P, U64, D, P, I64, P]),
            "cmbx_ensemble_create": (I, [ctypes.POINTER(_Job), I, I, ctypes.POINTER(P)]),
            "cmbx_ensemble_modes": (I, [P, ctypes.POINTER(I), I]),
            "cmbx_ensemble_lanes": (I, [P]),
            "cmbx_noise_tables": (I, [P, I]),
            "cmbx_ensemble_launch": (I, [P, P]),
            "cmbx_ensemble_destroy": (I, [P]),
            "cmbx_debug_noise": (I, [P, U64, P]),
            "cmbx_debug_field": (I, [P, U64, P]),
            "cmbx_debug_gather": (I, [P, P, D, P, I64, P]),
            "cmbx_footprint_bytes": (I64, [I]),
            "cmbx_healpix_cap": (I, [I64, D, P, I64, ctypes.POINTER(I64), P]),
            "cmbx_pixel_covariance": (I, [P, I64, P, I, P, P]),
            "cmbx_plan_autotune_patch": (I, [P, I, D, P, I64, P, P]),
            "cmbx_debug_footprint": (I, [P, D, P, I64, P]),
            "cmbx_debug_passes": (I, [P, U64, I, P]),
            "cmbx_time_passes": (I, [P, U64, D, P, I64, P, I, ctypes.POINTER(D)]),
            "cmbx_plan_autotune": (I, [P, I, ctypes.POINTER(I), ctypes.POINTER(D)]),
            "cmbx_tile_choices": (I, [I, I, I, ctypes.POINTER(I)]),
            "cmbx_enqueue_stage": (I, [P, I, U64, P, D, P, I64, P, P]),
            "cmbx_mlp_gemm": (I, [I, I, I, P, I, I, P, I, I, I, P, I, P, I, P, I, P]),
            "cmbx_mlp_gelu_backward": (I, [P, P, P, I64, P]),
            "cmbx_mlp_colsum": (I, [P, I, I, P, P]),
            "cmbx_mlp_mse": (I, [P, P, I64, P, P, P, P]),
            "cmbx_mlp_mse_partials": (I64, [I64]),
            "cmbx_mlp_mse_noalloc": (I, [P, P, I64, P, P, P]),
            "cmbx_mlp_adam": (I, [P, P, P, P, I64, ctypes.c_float, ctypes.c_float, ctypes.c_float,
                                  ctypes.c_float, I, P, P]),
            "cmbx_bf16_round": (I, [P, P, I64, P]),
            "cmbx_slab_create": (I, [I, I, I, I, D, I, I, ctypes.POINTER(P)]),
            "cmbx_slab_destroy": (I, [P]),
            "cmbx_slab_set": (I, [P, I, I64]),
            "cmbx_slab_observer": (I, [P, D, D, D]),
            "cmbx_slab_cap_observer": (I, [P, D, D, ctypes.POINTER(D)]),
            "cmbx_slab_spectrum": (I, [P, P, P, I64]),
            "cmbx_slab_simulate": (I, [P, U64, D, P, I64, P]),
            "cmbx_slab_debug_layers": (I, [P, U64, P]),
            "cmbx_slab_debug_columns": (I, [P, U64, P]),
            "cmbx_slab_factor": (I, [P, I64, P]),
            "cmbx_slab_info": (I, [P, ctypes.POINTER(I), ctypes.POINTER(I), ctypes.POINTER(I), ctypes.POINTER(D),
                                   ctypes.POINTER(P)]),
            "cmbx_box_size": (I, [D, D, D, D, ctypes.POINTER(I), ctypes.POINTER(I), ctypes.POINTER(D)]),
            "cmbx_cholesky": (I, [P, I64, I64, D, P, P]),
            "cmbx_whiten": (I, [P, I64, I64, P, I64, I64, P]),
            "cmbx_gemm_nt_sub": (I, [I64, I64, I, P, I64, P, I64, P, I64, I, P]),
            "cmbx_last_error": (ctypes.c_char_p, []),
            "cmbx_version": (ctypes.c_char_p, []),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype, f.argtypes = res, args
        _lib = L
    return _lib


def _check(rc):
    if rc != OK:
        raise CmbxError(rc, lib().cmbx_last_error().decode())
    return rc


def last_error():
    return lib().cmbx_last_error().decode()


def version():
    return lib().cmbx_version().decode()


def _ptr(x, nbytes=None, dtype=None, what="buffer"):
    """Device address of a torch CUDA tensor (checked) or a raw integer address."""
    if x is None:
        return None
    if isinstance(x, int):
        return x
    if not x.is_cuda:
        raise ValueError(f"{what} must be a CUDA tensor")
    if not x.is_contiguous():
        raise ValueError(f"{what} must be contiguous")
    if dtype is not None and x.dtype != dtype:
        raise ValueError(f"{what} must have dtype {dtype}, got {x.dtype}")
    if nbytes is not None and x.numel() * x.element_size() < nbytes:
        raise ValueError(f"{what} holds {x.numel() * x.element_size()} bytes, needs {nbytes}")
    return x.data_ptr()


# ------------------------------------------------------------------ raw ABI mirrors
def plan_box(N, L, dtype, batch):
    h = ctypes.c_void_p()
    _check(lib().cmbx_plan_box(int(N), float(L), _DTYPES[dtype], int(batch), ctypes.byref(h)))
    return h.value


def plan_destroy(h):
    return _check(lib().cmbx_plan_destroy(h))


def plan_set(h, key, value):
    return _check(lib().cmbx_plan_set(h, int(key), int(value)))


def plan_get(h, key):
    v = ctypes.c_int64(0)
    _check(lib().cmbx_plan_get(h, int(key), ctypes.byref(v)))
    return v.value


def spectrum_table(h, k, p_inf):
    k = np.ascontiguousarray(k, dtype=np.float64)
    p = np.ascontiguousarray(p_inf, dtype=np.float64)
    if k.shape != p.shape or k.ndim != 1:
        raise ValueError("k and P_inf must be 1-D arrays of equal length")
    return _check(lib().cmbx_spectrum_table(h, k.ctypes.data, p.ctypes.data, k.size))


def simulate_patch(h, seed, r, dirs, n_pix, out):
    return _check(lib().cmbx_simulate_patch(h, int(seed), float(r), dirs, int(n_pix), out))


def debug_noise(h, seed, halfgrid):
    return _check(lib().cmbx_debug_noise(h, int(seed), halfgrid))


def debug_field(h, seed, field):
    return _check(lib().cmbx_debug_field(h, int(seed), field))


def debug_gather(h, field, r, dirs, n_pix, out):
    return _check(lib().cmbx_debug_gather(h, field, float(r), dirs, int(n_pix), out))


# ------------------------------------------------------------------ owners
def healpix_cap_count(nside, z_min):
    """Pixels of the HEALPix (RING) cap of resolution nside holding the rings with z >= z_min
    (host only)."""
    n = ctypes.c_int64(0)
    _check(lib().cmbx_healpix_cap(int(nside), float(z_min), None, 0, ctypes.byref(n), None))
    return n.value


def healpix_cap(nside, z_min, out=None, stream=None):
    """Unit directions of that cap's pixels in RING order, made on the device: a
    [n_pix, 3] float64 CUDA tensor (`out` if given, with room for them)."""
    import torch
    n = healpix_cap_count(nside, z_min)
    if out is None:
        out = torch.empty((n, 3), dtype=torch.float64, device="cuda")
    if out.dim() != 2 or out.shape[1] != 3:
        raise ValueError("out must be a [n_pix, 3] float64 CUDA tensor")
    d = _ptr(out, n * 24, torch.float64, "out")
    if n == 0:
        return out[:0]
    s = stream if stream is not None else torch.cuda.current_stream().cuda_stream
    cnt = ctypes.c_int64(0)
    _check(lib().cmbx_healpix_cap(int(nside), float(z_min), d, out.shape[0], ctypes.byref(cnt), s))
    return out[:n]


def pixel_covariance(dirs, cl, out=None, stream=None):
    """Covariance [n_pix, n_pix] (float64 CUDA tensor) of maps with spectrum cl (l = 0 ..
    len(cl) - 1) at the unit directions dirs ([n_pix, 3] float64 CUDA tensor)."""
    import torch
    if dirs.dim() != 2 or dirs.shape[1] != 3:
        raise ValueError("dirs must be a [n_pix, 3] float64 CUDA tensor")
    n = dirs.shape[0]
    cl = torch.as_tensor(cl, dtype=torch.float64, device=dirs.device).contiguous()
    if out is None:
        out = torch.empty((n, n), dtype=torch.float64, device=dirs.device)
    d = _ptr(dirs, n * 24, torch.float64, "dirs")
    g = _ptr(out, n * n * 8, torch.float64, "out")
    s = stream if stream is not None else torch.cuda.current_stream().cuda_stream
    _check(lib().cmbx_pixel_covariance(d, n, cl.data_ptr(), cl.numel() - 1, g, s))
    return out


def cholesky(A, shift=0.0, stream=None):
    """In place: the lower triangle of A (n x n float64 CUDA tensor) becomes the Cholesky
    factor of A + shift I (cmbx_cholesky). Returns the device info word (int64 tensor of
    one element): 0, or the 1-based column of the first non-positive pivot."""
    import torch
    if A.dim() != 2 or A.shape[0] != A.shape[1]:
        raise ValueError("A must be a square matrix")
    n = A.shape[0]
    a = _ptr(A, n * n * 8, torch.float64, "A")
    info = torch.zeros(1, dtype=torch.int64, device=A.device)
    s = stream if stream is not None else torch.cuda.current_stream().cuda_stream
    _check(lib().cmbx_cholesky(a, n, n, float(shift), info.data_ptr(), s))
    return info


def whiten(L, maps, stream=None):
    """In place: every row m of maps (n_maps x n float64 CUDA tensor) becomes L^-1 m, L the
    lower triangle of the n x n tensor L (cmbx_whiten)."""
    import torch
    n = L.shape[0]
    if maps.dim() != 2 or maps.shape[1] != n:
        raise ValueError("maps must be (n_maps, n)")
    l = _ptr(L, n * n * 8, torch.float64, "L")
    b = _ptr(maps, maps.numel() * 8, torch.float64, "maps")
    s = stream if stream is not None else torch.cuda.current_stream().cuda_stream
    _check(lib().cmbx_whiten(l, n, n, b, maps.shape[0], n, s))
    return maps


class Plan:
    """A box plan (N^3, side L, precision, batch) bound to a stream.

    ``stream``: a torch.cuda.Stream, a raw hipStream_t integer, or None for torch's
    current stream (so the plan's work is ordered with torch's allocations).
    ``prune``: maps are made from only the part of the field their stencils read (the
    same maps; the workspace then holds only that part of the field).
    """

    def __init__(self, N, L=1.0, dtype="f32", batch=1, interp="trilinear", stream=None, prune=True):
        import torch
        self.N, self.L, self.batch = int(N), float(L), int(batch)
        self.dtype = _DTYPES[dtype]
        self.torch_dtype = torch.float32 if self.dtype == F32 else torch.float64
        self.handle = plan_box(N, L, self.dtype, batch)
        try:
            self.set_interp(interp)
            self.set_prune(prune)
            if stream is None:
                stream = torch.cuda.current_stream()
            self.stream = stream
            plan_set(self.handle, OPT_STREAM, stream if isinstance(stream, int) else stream.cuda_stream)
        except Exception:
            self.close()
            raise

    def close(self):
        if getattr(self, "handle", None):
            plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_observer(self, position):
        """Observer position (x, y, z) in the box, units of L (default: the centre)."""
        x, y, z = (float(v) for v in position)
        _check(lib().cmbx_plan_observer(self.handle, x, y, z))
        self.observer = (x, y, z)

    def observer_for_cap(self, r, z_min):
        """The position that centres the box on the cap about +z at radius r whose edge is
        z_min (cmbx_plan_cap_observer)."""
        xyz = (ctypes.c_double * 3)()
        _check(lib().cmbx_plan_cap_observer(self.handle, float(r), float(z_min), xyz))
        return tuple(xyz)

    def set_prune(self, prune):
        self.prune = bool(prune)
        plan_set(self.handle, OPT_PRUNE, int(self.prune))

    def set_fixed_dirs(self, fixed=True):
        """CMBX_OPT_FIXED_DIRS: reuse the map footprint while (r, dirs, n_pix, ...) repeat; call
        again after writing new directions into the same tensor."""
        self.fixed_dirs = bool(fixed)
        plan_set(self.handle, OPT_FIXED_DIRS, int(self.fixed_dirs))

    def set_interp(self, interp):
        self.interp = _INTERPS[interp]
        plan_set(self.handle, OPT_INTERP, self.interp)

    def set_tiles(self, tile_xy=0, lines_z=0, tile_x=None, tile_y=None, plans=None):
        """Workgroup tile shapes (0 = compiled default); tile_x / tile_y override tile_xy;
        plans = (x, y, z) FFT stage plans (0 or 1; plan 1 at the default tiles only)."""
        plan_set(self.handle, OPT_TILE_XY, tile_xy)
        if tile_x is not None:
            plan_set(self.handle, OPT_TILE_X, tile_x)
        if tile_y is not None:
            plan_set(self.handle, OPT_TILE_Y, tile_y)
        plan_set(self.handle, OPT_LINES_Z, lines_z)
        for key, v in zip((OPT_PLAN_X, OPT_PLAN_Y, OPT_PLAN_Z), plans or (0, 0, 0)):
            plan_set(self.handle, key, v)

    def shapes(self):
        """(tile_x, tile_y, lines_z, (plan_x, plan_y, plan_z)) in use."""
        g = lambda k: plan_get(self.handle, k)  # noqa: E731
        return g(OPT_TILE_X), g(OPT_TILE_Y), g(OPT_LINES_Z), (g(OPT_PLAN_X), g(OPT_PLAN_Y), g(OPT_PLAN_Z))

    def spectrum_table(self, k, p_inf):
        spectrum_table(self.handle, k, p_inf)

    def autotune(self, reps=5, cache_path=None, use_cache=True, r=None, dirs=None):
        """Choose the tile shapes and FFT stage plans of the three field kernels whose
        x -> y -> z chain runs fastest (timed on the device by cmbx_plan_autotune) and
        remember them in a JSON cache keyed by (arch, N, precision, tuning rule). A cached
        entry is reused if every value is still a compiled choice; otherwise the plan is
        re-tuned. Returns dict(tile_x, tile_y, lines_z, plans, ms) with ms the time of each
        pass alone.

        With ``r`` and ``dirs`` (a map's pixels) a pruning plan is tuned on the passes as
        that map makes them (cmbx_plan_autotune_patch); the choice depends on the map's
        footprint, so it is not cached."""
        import json
        path = cache_path or TUNE_CACHE
        key = f"gfx950:N{self.N}:{'f32' if self.dtype == F32 else 'f64'}:chain+plans"
        patch = dirs is not None and self.prune
        if patch:
            if r is None:
                raise ValueError("autotune with dirs needs r")
            import torch
            use_cache = False
            d = _ptr(dirs, dirs.shape[0] * 24, torch.float64, "dirs")
        cache = _load_cache(path) if use_cache else {}
        ent = cache.get(key)
        txy = tile_choices(self.dtype, self.N, 0)
        tz = tile_choices(self.dtype, self.N, 1)
        if (isinstance(ent, dict) and ent.get("tile_x") in txy and ent.get("tile_y") in txy
                and ent.get("lines_z") in tz and isinstance(ent.get("plans"), list) and len(ent["plans"]) == 3):
            try:
                self.set_tiles(0, ent["lines_z"], tile_x=ent["tile_x"], tile_y=ent["tile_y"], plans=ent["plans"])
                return dict(ent, cached=True)
            except CmbxError:
                pass  # a plan no longer compiled: tune again
        best = (ctypes.c_int * 3)()
        ms = (ctypes.c_double * 3)()
        if patch:
            _check(lib().cmbx_plan_autotune_patch(self.handle, int(reps), float(r), d, int(dirs.shape[0]), best, ms))
        else:
            _check(lib().cmbx_plan_autotune(self.handle, int(reps), best, ms))
        tx, ty, lz, plans = self.shapes()
        ent = {"tile_x": tx, "tile_y": ty, "lines_z": lz, "plans": list(plans), "ms": list(ms)}
        if use_cache:
            cache[key] = ent
            try:
                os.makedirs(os.path.dirname(path), exist_ok=True)
                tmp = path + ".tmp"
                with open(tmp, "w") as f:
                    json.dump(cache, f, indent=1)
                os.replace(tmp, path)
            except OSError:
                pass
        return dict(ent, cached=False)

    @property
    def real_size(self):
        return 4 if self.dtype == F32 else 8

    def field_ptr(self, b=0):
        f = ctypes.c_void_p()
        _check(lib().cmbx_plan_info(self.handle, None, None, None, None, ctypes.byref(f)))
        return f.value + b * self.N**3 * self.real_size

    def field(self, b=0):
        """A copy of realisation b's field from the plan's workspace, [N][N][N] tensor (after
        simulate_patch on a pruning plan only the part the map's stencils read is valid)."""
        import torch
        out = torch.empty((self.N, self.N, self.N), dtype=self.torch_dtype, device="cuda")
        _memcpy_d2d(out.data_ptr(), self.field_ptr(b), self.N**3 * self.real_size, self.stream)
        return out

    def _check_dirs_out(self, dirs, out, n_pix=None):
        import torch
        if n_pix is None:
            n_pix = dirs.shape[0] if not isinstance(dirs, int) else None
        if n_pix is None:
            raise ValueError("n_pix is required with raw pointers")
        if not isinstance(dirs, int) and (dirs.dim() != 2 or dirs.shape[1] != 3 or dirs.shape[0] < n_pix):
            raise ValueError("dirs must be a [n_pix, 3] float64 CUDA tensor")
        d = _ptr(dirs, n_pix * 24, torch.float64, "dirs")
        o = _ptr(out, self.batch * n_pix * self.real_size, self.torch_dtype, "out")
        return d, o, n_pix

    def simulate_patch(self, seed, r, dirs, out=None, n_pix=None):
        """Maps [batch, n_pix] of realisations seed .. seed + batch - 1."""
        import torch
        if out is None:
            n = dirs.shape[0]
            out = torch.empty((self.batch, n), dtype=self.torch_dtype, device="cuda")
        d, o, n_pix = self._check_dirs_out(dirs, out, n_pix)
        simulate_patch(self.handle, seed, r, d, n_pix, o)
        return out

    def time_passes(self, seed, r, dirs, out, reps=10):
        """Average ms of (pass x, pass y, pass z, gather) over ``reps`` launches each."""
        d, o, n_pix = self._check_dirs_out(dirs, out)
        ms = (ctypes.c_double * 4)()
        _check(lib().cmbx_time_passes(self.handle, int(seed), float(r), d, n_pix, o, int(reps), ms))
        return list(ms)

    def enqueue_stage(self, stage, seed, buf, r=0.0, dirs=None, out=None, stream=None):
        """One stage (0 noise + x, 1 y, 2 z, 3 gather) of realisation ``seed`` on ``buf``."""
        b = _ptr(buf, self.N**3 * self.real_size, self.torch_dtype, "buf")
        d = o = None
        n_pix = 0
        if stage == 3:
            d, o, n_pix = self._check_dirs_out(dirs, out)
        s = 0 if stream is None else (stream if isinstance(stream, int) else stream.cuda_stream)
        _check(lib().cmbx_enqueue_stage(self.handle, int(stage), int(seed), b, float(r), d, int(n_pix), o, s))

    def debug_noise(self, seed):
        import torch
        ctype = torch.complex64 if self.dtype == F32 else torch.complex128
        h = torch.empty((self.N, self.N, self.N // 2 + 1), dtype=ctype, device="cuda")
        debug_noise(self.handle, seed, h.data_ptr())
        return h

    def debug_field(self, seed):
        import torch
        f = torch.empty((self.N, self.N, self.N), dtype=self.torch_dtype, device="cuda")
        debug_field(self.handle, seed, f.data_ptr())
        return f

    def debug_passes(self, seed, npasses):
        """Workspace after the first ``npasses`` kernels: complex [N][N][N/2] for 1-2 passes,
        real [N][N][N] after 3. The kernels leave entries that the spectrum's support makes
        zero unwritten; the buffer starts zeroed, so they read as that zero."""
        import torch
        ctype = torch.complex64 if self.dtype == F32 else torch.complex128
        if npasses < 3:
            b = torch.zeros((self.N, self.N, self.N // 2), dtype=ctype, device="cuda")
        else:
            b = torch.zeros((self.N, self.N, self.N), dtype=self.torch_dtype, device="cuda")
        _check(lib().cmbx_debug_passes(self.handle, int(seed), int(npasses), b.data_ptr()))
        return b

    def debug_footprint(self, r, dirs, out=None):
        """The map footprint of (r, dirs) as simulate_patch makes it on a pruning plan:
        (planes [N] uint8, blocks [N][ceil(N/8)] uint8, zblocks [ceil(N/32)] uint8, lines,
        sorted z-block list, sorted plane list) as numpy arrays; the raw device buffer goes
        to `out` if given (uint8 tensor)."""
        import numpy as np
        import torch
        nbytes = int(lib().cmbx_footprint_bytes(self.N))
        if nbytes < 0:
            _check(nbytes)
        if out is None:
            out = torch.zeros(nbytes, dtype=torch.uint8, device="cuda")
        _check(lib().cmbx_debug_footprint(self.handle, float(r), dirs.data_ptr(), int(dirs.shape[0]), out.data_ptr()))
        raw = out.cpu().numpy()
        N, nb, nzb = self.N, (self.N + 7) // 8, (self.N + 31) // 32
        zoff = N * (1 + nb)
        off = (zoff + nzb + 3) // 4 * 4
        hdr = raw[off:off + 16].view(np.uint32)
        zl = off + 16
        pl = zl + 4 * N * N
        zlist = raw[zl:zl + 4 * int(hdr[1])].view(np.uint32)
        plist = raw[pl:pl + 4 * int(hdr[2])].view(np.uint32)
        return (raw[:N].copy(), raw[N:zoff].reshape(N, nb).copy(), raw[zoff:zoff + nzb].copy(), int(hdr[0]),
                np.sort(zlist), np.sort(plist))

    def debug_gather(self, field, r, dirs, out=None):
        import torch
        n = dirs.shape[0]
        if out is None:
            out = torch.empty((n,), dtype=self.torch_dtype, device="cuda")
        fp = _ptr(field, self.N**3 * self.real_size, self.torch_dtype, "field")
        d = _ptr(dirs, n * 24, torch.float64, "dirs")
        o = _ptr(out, n * self.real_size, self.torch_dtype, "out")
        debug_gather(self.handle, fp, r, d, n, o)
        return out


def tile_choices(dtype, N, which):
    """Compiled tile choices: which = 0 (x/y column tiles) or 1 (z lines)."""
    out = (ctypes.c_int * 4)()
    n = lib().cmbx_tile_choices(_DTYPES[dtype], int(N), int(which), out)
    return list(out[:n])


TUNE_CACHE = os.environ.get("CMBX_TUNE_CACHE", os.path.join(os.path.expanduser("~"), ".cache", "cmbx", "tune.json"))


def _load_cache(path):
    import json
    try:
        with open(path) as f:
            data = json.load(f)
        return data if isinstance(data, dict) else {}
    except (OSError, ValueError):
        return {}  # missing or corrupt cache: start afresh


def _memcpy_d2d(dst, src, nbytes, stream):
    hip = _hip()
    s = stream if isinstance(stream, int) else stream.cuda_stream
    rc = hip.hipMemcpyAsync(ctypes.c_void_p(dst), ctypes.c_void_p(src), ctypes.c_size_t(nbytes), 3, ctypes.c_void_p(s))
    if rc != 0:
        raise RuntimeError(f"hipMemcpyAsync failed ({rc})")


_hip_rt = None


def _hip():
    global _hip_rt
    if _hip_rt is None:
        _hip_rt = ctypes.CDLL("libamdhip64.so")
        _hip_rt.hipMemcpyAsync.restype = ctypes.c_int
    return _hip_rt


class Ensemble:
    """Jobs captured into one HIP graph (cmbx_ensemble_create)."""

    _MODES = {"auto": ENS_AUTO, "chained": ENS_CHAINED, "pipelined": ENS_PIPELINED}

    def __init__(self, jobs, mode="auto", lanes=None):
        """jobs: list of dict(plan=Plan, seed, r, dirs=tensor, out=tensor). lanes: None
        (auto mode times 1 .. 4 lanes; explicit modes use one) or 1 .. 4."""
        arr = (_Job * len(jobs))()
        self._keep = []
        for i, j in enumerate(jobs):
            p = j["plan"]
            d, o, n_pix = p._check_dirs_out(j["dirs"], j["out"])
            arr[i] = _Job(p.handle, int(j["seed"]), float(j["r"]), d, n_pix, o)
            self._keep.append(j)
        h = ctypes.c_void_p()
        if lanes is not None and not 1 <= int(lanes) <= ENS_MAX_LANES:
            raise ValueError(f"lanes must be 1 .. {ENS_MAX_LANES}")
        flags = 0 if lanes is None else int(lanes) << 8
        _check(lib().cmbx_ensemble_create(arr, len(jobs), self._MODES.get(mode, mode) | flags, ctypes.byref(h)))
        self.handle = h.value

    @property
    def modes(self):
        """Execution mode per (precision, N) group: "chained" or "pipelined"."""
        buf = (ctypes.c_int * 64)()
        n = lib().cmbx_ensemble_modes(self.handle, buf, 64)
        names = {ENS_CHAINED: "chained", ENS_PIPELINED: "pipelined"}
        return [names.get(buf[i], buf[i]) for i in range(min(n, 64))]

    @property
    def lanes(self):
        """Number of graphs (and streams) the ensemble runs in."""
        n = lib().cmbx_ensemble_lanes(self.handle)
        if n < 0:
            _check(n)
        return n

    def launch(self, stream=None):
        import torch
        if stream is None:
            stream = torch.cuda.current_stream()
        s = stream if isinstance(stream, int) else stream.cuda_stream
        _check(lib().cmbx_ensemble_launch(self.handle, s))

    def close(self):
        if getattr(self, "handle", None):
            _check(lib().cmbx_ensemble_destroy(self.handle))
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def box_size(b, theta_max, size_factor=1.0, R=1.0):
    """The box sizing rule of Sec. II C (cmbx_box_size): (N, M, dp) for beam b and cap
    half-angle theta_max (radians) on a sphere of radius R."""
    n, m, d = ctypes.c_int(), ctypes.c_int(), ctypes.c_double()
    _check(lib().cmbx_box_size(float(b), float(theta_max), float(size_factor), float(R), ctypes.byref(n),
                               ctypes.byref(m), ctypes.byref(d)))
    return n.value, m.value, d.value


class Slab:
    """Stacked layers of a flat N x N x M box (cmbx_slab_*): method "flat" (the 3-D Fourier
    method on the whole box, nz = M layers) or "hybrid" (the 2-D Fourier method, h layers).
    Lengths (dp, r, observer) share one unit."""

    _METHODS = {"flat": SLAB_FLAT, "hybrid": SLAB_HYBRID, SLAB_FLAT: SLAB_FLAT, SLAB_HYBRID: SLAB_HYBRID}

    def __init__(self, method, N, M, dp, h=None, dtype="f32", batch=1, interp="trilinear", stream=None):
        import torch
        self.method = self._METHODS[method]
        self.N, self.M, self.dp, self.batch = int(N), int(M), float(dp), int(batch)
        self.dtype = _DTYPES[dtype]
        self.torch_dtype = torch.float32 if self.dtype == F32 else torch.float64
        hh = self.M if self.method == SLAB_FLAT else int(h)
        handle = ctypes.c_void_p()
        _check(lib().cmbx_slab_create(self.method, self.N, self.M, hh, self.dp, self.dtype, self.batch,
                                      ctypes.byref(handle)))
        self.handle = handle.value
        try:
            nz = ctypes.c_int()
            _check(lib().cmbx_slab_info(self.handle, None, None, ctypes.byref(nz), None, None))
            self.nz = nz.value
            self.set_interp(interp)
            if stream is None:
                stream = torch.cuda.current_stream()
            self.stream = stream
            _check(lib().cmbx_slab_set(self.handle, OPT_STREAM, stream if isinstance(stream, int) else stream.cuda_stream))
        except Exception:
            self.close()
            raise

    def close(self):
        if getattr(self, "handle", None):
            _check(lib().cmbx_slab_destroy(self.handle))
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_interp(self, interp):
        self.interp = _INTERPS[interp]
        _check(lib().cmbx_slab_set(self.handle, OPT_INTERP, self.interp))

    def set_direct(self, mode):
        """How maps take their values from the layers: "always" sums each stencil row
        directly from its line's half spectrum after the transform along x, "never" runs
        the complex-to-real pass and the gather, "auto" (default) sums directly for few
        pixels (CMBX_SLAB_OPT_DIRECT)."""
        _check(lib().cmbx_slab_set(self.handle, SLAB_OPT_DIRECT, _DIRECT[mode]))

    def set_observer(self, position):
        x, y, z = (float(v) for v in position)
        _check(lib().cmbx_slab_observer(self.handle, x, y, z))
        self.observer = (x, y, z)

    def observer_for_cap(self, r, z_min):
        """The middle of the layers at the middle height of the cap about +z of radius r and
        edge z_min (cmbx_slab_cap_observer)."""
        xyz = (ctypes.c_double * 3)()
        _check(lib().cmbx_slab_cap_observer(self.handle, float(r), float(z_min), xyz))
        return tuple(xyz)

    def spectrum(self, k, p_inf):
        k = np.ascontiguousarray(k, dtype=np.float64)
        p = np.ascontiguousarray(p_inf, dtype=np.float64)
        if k.shape != p.shape or k.ndim != 1:
            raise ValueError("k and P_inf must be 1-D arrays of equal length")
        _check(lib().cmbx_slab_spectrum(self.handle, k.ctypes.data, p.ctypes.data, k.size))

    def simulate(self, seed, r, dirs, out=None):
        """Maps [batch, n_pix] of realisations seed .. seed + batch - 1."""
        import torch
        if dirs.dim() != 2 or dirs.shape[1] != 3:
            raise ValueError("dirs must be a [n_pix, 3] float64 CUDA tensor")
        n = dirs.shape[0]
        if out is None:
            out = torch.empty((self.batch, n), dtype=self.torch_dtype, device="cuda")
        d = _ptr(dirs, n * 24, torch.float64, "dirs")
        o = _ptr(out, self.batch * n * (4 if self.dtype == F32 else 8), self.torch_dtype, "out")
        _check(lib().cmbx_slab_simulate(self.handle, int(seed), float(r), d, n, o))
        return out

    def debug_layers(self, seed):
        import torch
        out = torch.empty((self.nz, self.N, self.N), dtype=self.torch_dtype, device="cuda")
        _check(lib().cmbx_slab_debug_layers(self.handle, int(seed), out.data_ptr()))
        return out

    def debug_columns(self, seed):
        """Flat: the modes [N][N/2+1][M]; hybrid: the correlated columns [h][N][N/2+1]."""
        import torch
        ctype = torch.complex64 if self.dtype == F32 else torch.complex128
        shape = (self.N, self.N // 2 + 1, self.M) if self.method == SLAB_FLAT else (self.nz, self.N, self.N // 2 + 1)
        out = torch.empty(shape, dtype=ctype, device="cuda")
        _check(lib().cmbx_slab_debug_columns(self.handle, int(seed), out.data_ptr()))
        return out

    def factor(self, s):
        """FP64 factor S (h x h) of the columns with fx^2 + fy^2 = s (hybrid)."""
        out = np.empty((self.nz, self.nz), dtype=np.float64)
        _check(lib().cmbx_slab_factor(self.handle, int(s), out.ctypes.data))
        return out
