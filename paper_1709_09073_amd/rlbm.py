"""Thin ctypes binding of librlbm.so (include/rlbm.h): argument marshalling only.

Every step of the method runs in the HIP kernels; PyTorch provides the device
buffers and the stream.  Importing this module loads the library and fails loudly
if it has not been built (python -m paper_1709_09073_amd.build).
"""
import ctypes
import os

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "librlbm.so")

RLBM_OK, RLBM_EINVAL, RLBM_EDOMAIN, RLBM_EHIP, RLBM_ENONFINITE, RLBM_ENOTIMPL = 0, -1, -2, -3, -4, -5
STATS = {"MJ": 0, "FD": 1, "BE": 2}
PRECISION = {"fp64": 0, "fp32": 1, "dev16": 2}
TAU_MODE = {"const": 0, "theta": 1}
BC = {"periodic": 0, "open": 1, "wall": 2, "wall_neq": 3}
GUESS = {"fixed": 0, "mlp": 1}
DTYPE = {"fp64": torch.float64, "fp32": torch.float32}
DEV16_BYTES_PER_CELL = 192   # 72 SNORM16 deviations + 8 float side values + 6 half scales + padding
FIELD_NAMES = ("n", "eps", "theta", "z", "ux", "uy", "qx", "qy")
MOMENT_NAMES = ("N0", "Nx", "Ny", "T00", "T0x", "T0y", "Txx", "Txy", "Tyy")

FLAG_NONPOSITIVE, FLAG_SUPERLUMINAL, FLAG_CONDENSED, FLAG_RANGE, FLAG_NOCONV = 0x1, 0x2, 0x4, 0x8, 0x10
FLAG_NONFINITE, FLAG_UNSTABLE = 0x20, 0x40
MLP_HIDDEN = 32
MLP_FLOATS = 4 + 3 * MLP_HIDDEN + 1
MLP_NTRAIN = 3 * MLP_HIDDEN + 1
MLP_NOALLOC_MAX = 32768   # samples the allocation-free training call accepts


class Params(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("stats", ctypes.c_int32),
                ("order", ctypes.c_int32), ("precision", ctypes.c_int32), ("tau_mode", ctypes.c_int32),
                ("tau", ctypes.c_double), ("tau_a", ctypes.c_double), ("tau_b", ctypes.c_double),
                ("bc", ctypes.c_int32 * 4), ("theta_wall", ctypes.c_double * 2), ("guess", ctypes.c_int32),
                ("mlp", ctypes.c_void_p), ("f_a", ctypes.c_void_p), ("f_b", ctypes.c_void_p),
                ("stream", ctypes.c_void_p), ("tile_x", ctypes.c_int32), ("tile_y", ctypes.c_int32),
                ("collect_stats", ctypes.c_int32), ("force", ctypes.c_double * 2), ("wall_n", ctypes.c_double),
                ("wall_theta", ctypes.c_double), ("check", ctypes.c_int32)]


class InitFields(ctypes.Structure):
    _fields_ = [("n", ctypes.c_void_p), ("z", ctypes.c_void_p), ("theta", ctypes.c_void_p),
                ("ux", ctypes.c_void_p), ("uy", ctypes.c_void_p), ("given_z", ctypes.c_int32)]


class OutFields(ctypes.Structure):
    _fields_ = [(k, ctypes.c_void_p) for k in FIELD_NAMES + MOMENT_NAMES]


class RlbmError(RuntimeError):
    def __init__(self, code, what=""):
        self.code = code
        super().__init__(f"{what}: {lib().rlbm_strerror(code).decode()} ({code})")


_LIB = None


def lib():
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_1709_09073_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        L.rlbm_init.argtypes = [ctypes.POINTER(ctypes.c_void_p), ctypes.POINTER(Params), ctypes.POINTER(InitFields)]
        L.rlbm_step.argtypes = [ctypes.c_void_p, ctypes.c_int64]
        L.rlbm_moments.argtypes = [ctypes.c_void_p, ctypes.POINTER(OutFields)]
        L.rlbm_state_index.argtypes = [ctypes.c_void_p]
        L.rlbm_steps_done.argtypes = [ctypes.c_void_p]
        L.rlbm_steps_done.restype = ctypes.c_int64
        L.rlbm_sync.argtypes = [ctypes.c_void_p]
        L.rlbm_status.argtypes = [ctypes.c_void_p]
        L.rlbm_status.restype = ctypes.c_uint32
        L.rlbm_free.argtypes = [ctypes.c_void_p]
        L.rlbm_free.restype = None
        L.rlbm_strerror.argtypes = [ctypes.c_int]
        L.rlbm_strerror.restype = ctypes.c_char_p
        L.rlbm_init_batch.argtypes = [ctypes.POINTER(ctypes.c_void_p), ctypes.c_int32, ctypes.POINTER(Params),
                                      ctypes.POINTER(InitFields)]
        L.rlbm_autotune.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32),
                                    ctypes.POINTER(ctypes.c_int32)]
        L.rlbm_capture.argtypes = [ctypes.c_void_p]
        L.rlbm_configure.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32]
        L.rlbm_moments_grid.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(OutFields)]
        L.rlbm_inversion_stats.argtypes = [ctypes.c_void_p, ctypes.POINTER(ctypes.c_uint64), ctypes.POINTER(ctypes.c_uint64)]
        L.rlbm_inversion_samples.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
        L.rlbm_noneq_tensors.argtypes = [ctypes.c_void_p, ctypes.c_int32] + [ctypes.c_void_p] * 4
        L.rlbm_mlp_workspace_bytes.argtypes = [ctypes.c_int64]
        L.rlbm_mlp_workspace_bytes.restype = ctypes.c_uint64
        vp = ctypes.c_void_p
        L.rlbm_mlp_init.argtypes = [vp, vp, vp, ctypes.c_int64, vp, vp, vp]
        L.rlbm_mlp_loss_grad.argtypes = [vp, vp, vp, ctypes.c_int64, vp, vp, vp, vp]
        L.rlbm_mlp_train.argtypes = [vp, vp, vp, ctypes.c_int64, ctypes.c_int32, ctypes.c_float, vp, vp, vp]
        L.rlbm_mlp_predict.argtypes = [vp, vp, vp, ctypes.c_int64, vp]
        L.rlbm_mlp_train_noalloc.argtypes = [vp, vp, vp, ctypes.c_int64, ctypes.c_int32, ctypes.c_float, vp, vp]
        _LIB = L
    return _LIB


def unpack_populations(buf, precision, nx, ny):
    """(72, ny, nx) populations, q = 6 n + k, from an FP32/FP64 buffer in the library's
    layout: per direction n a block of nx*ny cell records, FP32 shells 0..3 (16 bytes
    each cell) followed by shells 4..5 (8 bytes), FP64 shell pairs (0,1), (2,3),
    (4,5) as three runs of 16-byte records.  Returns a new tensor."""
    P = nx * ny
    blk = buf.reshape(12, 6 * P)
    if precision == "fp32":
        rec = torch.cat([blk[:, :4 * P].reshape(12, P, 4), blk[:, 4 * P:].reshape(12, P, 2)], dim=2)
    elif precision == "fp64":
        rec = blk.reshape(12, 3, P, 2).permute(0, 2, 1, 3).reshape(12, P, 6)
    else:
        raise ValueError("16-bit deviation buffers: use dev16_views")
    return rec.permute(0, 2, 1).reshape(72, ny, nx).contiguous()


def pack_populations(f, precision):
    """Inverse of unpack_populations: a flat buffer in the library's layout."""
    _, ny, nx = f.shape
    P = nx * ny
    rec = f.reshape(12, 6, P).permute(0, 2, 1)
    if precision == "fp32":
        out = torch.cat([rec[:, :, :4].reshape(12, 4 * P), rec[:, :, 4:].reshape(12, 2 * P)], dim=1)
    elif precision == "fp64":
        out = rec.reshape(12, P, 3, 2).permute(0, 2, 1, 3)
    else:
        raise ValueError("16-bit deviation buffers cannot be packed from populations")
    return out.reshape(-1).contiguous()


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def _check(code, what):
    if code != RLBM_OK:
        raise RlbmError(code, what)


def _grid_args(params, init, device, stream):
    """Population buffers, rlbm_params and rlbm_init_fields for one grid."""
    nx, ny = int(params["nx"]), int(params["ny"])
    prec = params.get("precision", "fp64")
    if prec == "dev16":
        f = [torch.empty(DEV16_BYTES_PER_CELL * nx * ny // 4, dtype=torch.float32, device=device) for _ in range(2)]
    else:
        f = [torch.empty(72 * nx * ny, dtype=DTYPE[prec], device=device) for _ in range(2)]
    bc = params.get("bc", ("periodic",) * 4)
    tw = params.get("theta_wall", (1.0, 1.0))
    p = Params(nx=nx, ny=ny, stats=STATS[params.get("stats", "MJ")], order=int(params.get("order", 5)),
               precision=PRECISION[prec], tau_mode=TAU_MODE[params.get("tau_mode", "const")],
               tau=float(params.get("tau", 1.0)), tau_a=float(params.get("tau_a", 2.0)),
               tau_b=float(params.get("tau_b", 0.2546)), guess=GUESS[params.get("guess", "fixed")],
               mlp=_ptr(params.get("mlp")), f_a=_ptr(f[0]), f_b=_ptr(f[1]),
               stream=ctypes.c_void_p(stream.cuda_stream),
               tile_x=int(params.get("tile", (0, 0))[0]), tile_y=int(params.get("tile", (0, 0))[1]),
               collect_stats=int(bool(params.get("collect_stats", False))),
               wall_n=float(params.get("wall_n", 1.0)), wall_theta=float(params.get("wall_theta", 1.0)),
               check=int(bool(params.get("check", False))))
    p.bc[:] = [BC[b] for b in bc]
    p.theta_wall[:] = [float(t) for t in tw]
    p.force[:] = [float(a) for a in params.get("force", (0.0, 0.0))]
    keep = {k: v.contiguous().to(device=device, dtype=torch.float64) for k, v in init.items()}
    fi = InitFields(n=_ptr(keep.get("n")), z=_ptr(keep.get("z")), theta=_ptr(keep["theta"]), ux=_ptr(keep["ux"]),
                    uy=_ptr(keep["uy"]), given_z=int("z" in keep))
    return f, p, fi, keep


class Sim:
    """One grid: owns two population tensors (ping-pong) on the current CUDA/HIP device.

    params: dict with keys nx, ny, stats ('MJ'|'FD'|'BE'), order (2..5, default 5),
    precision ('fp64'|'fp32'|'dev16'), tau_mode ('const'|'theta'), tau, tau_a, tau_b,
    bc (xlo, xhi, ylo, yhi names from BC), theta_wall (xlo, xhi), guess ('fixed'|'mlp')
    with mlp (the network's weight tensor), tile ((tile_x, tile_y), default automatic),
    collect_stats, force ((a_x, a_y), momentum update), wall_n and wall_theta (state
    imposed on 'wall_neq' sides), check (every step call waits and reports the status
    word).  init: dict of (ny, nx) float64 CUDA tensors theta, ux, uy and either n or z.
    """

    def __init__(self, params, init, device="cuda", stream=None):
        self.stream = stream if stream is not None else torch.cuda.current_stream(device)
        self.nx, self.ny = int(params["nx"]), int(params["ny"])
        self.precision = params.get("precision", "fp64")
        self.params = dict(params)
        self.f, self._p, self._fi, self._keep = _grid_args(params, init, device, self.stream)
        ctx = ctypes.c_void_p()
        _check(lib().rlbm_init(ctypes.byref(ctx), ctypes.byref(self._p), ctypes.byref(self._fi)), "rlbm_init")
        self.ctx = ctx

    def capture(self):
        """Capture the replayed step graphs now (no step is run)."""
        _check(lib().rlbm_capture(self.ctx), "rlbm_capture")

    def autotune(self, trial_steps=5):
        tx, ty = ctypes.c_int32(), ctypes.c_int32()
        _check(lib().rlbm_autotune(self.ctx, int(trial_steps), ctypes.byref(tx), ctypes.byref(ty)), "rlbm_autotune")
        return tx.value, ty.value

    def step(self, nsteps=1):
        _check(lib().rlbm_step(self.ctx, int(nsteps)), "rlbm_step")

    def state(self):
        """The buffer holding the current post-collision state (library layout)."""
        return self.f[lib().rlbm_state_index(self.ctx)]

    def populations(self):
        """Current post-collision populations as a (72, ny, nx) tensor (FP32/FP64)."""
        self.sync()
        return unpack_populations(self.state(), self.precision, self.nx, self.ny)

    def set_populations(self, f):
        """Overwrite the current state with populations f of shape (72, ny, nx)."""
        self.sync()
        st = self.state()
        st.copy_(pack_populations(f.to(device=st.device, dtype=st.dtype), self.precision))
        torch.cuda.synchronize(st.device)

    def load_state(self, saved):
        """Resume from a saved post-collision state (a tensor like state()): the
        populations are the whole state, so copying them into the current buffer
        restarts the run; the step counter is not part of the physics."""
        self.sync()
        self.state().copy_(saved)
        torch.cuda.synchronize(self.state().device)

    @property
    def steps_done(self):
        return lib().rlbm_steps_done(self.ctx)

    def fields(self, names=FIELD_NAMES, check=True):
        """Fields (and, if named, raw moments MOMENT_NAMES) of the current state."""
        out = {k: torch.empty((self.ny, self.nx), dtype=torch.float64, device=self.f[0].device) for k in names}
        of = OutFields(**{k: _ptr(out.get(k)) for k in FIELD_NAMES + MOMENT_NAMES})
        rc = lib().rlbm_moments(self.ctx, ctypes.byref(of))
        if check:
            _check(rc, "rlbm_moments")
        return out

    def noneq_tensors(self, check=True):
        """{r: pi^{x..x} of rank r} for r = 2..5 (float64 (ny, nx) tensors)."""
        out = {r: torch.empty((self.ny, self.nx), dtype=torch.float64, device=self.f[0].device) for r in (2, 3, 4, 5)}
        rc = lib().rlbm_noneq_tensors(self.ctx, 0, *(_ptr(out[r]) for r in (2, 3, 4, 5)))
        if check:
            _check(rc, "rlbm_noneq_tensors")
        return out

    def sync(self):
        _check(lib().rlbm_sync(self.ctx), "rlbm_sync")

    def inversion_stats(self):
        it, so = ctypes.c_uint64(), ctypes.c_uint64()
        _check(lib().rlbm_inversion_stats(self.ctx, ctypes.byref(it), ctypes.byref(so)), "rlbm_inversion_stats")
        return it.value, so.value

    def inversion_samples(self):
        """(x, t) float32 tensors (ny, nx): x = ln(2 n^3 / (pi eps^2)), t = ln z."""
        dev = self.f[0].device
        x = torch.empty((self.ny, self.nx), dtype=torch.float32, device=dev)
        t = torch.empty_like(x)
        _check(lib().rlbm_inversion_samples(self.ctx, _ptr(x), _ptr(t)), "rlbm_inversion_samples")
        return x, t

    def status(self):
        return lib().rlbm_status(self.ctx)

    def close(self):
        if getattr(self, "ctx", None):
            lib().rlbm_free(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def dev16_views(buf, nx, ny):
    """(deviations (72, ny, nx) int16 with q = 6 n + k, side values (8, ny, nx) float32
    rho_0..rho_5, alpha, beta, shell scales (6, ny, nx) float16) of an RLBM_DEV16 buffer,
    rearranged from its cell-packed layout (12 direction blocks of cells x 6 SNORM16,
    then cells x 48-byte side records); copies."""
    raw = buf.view(torch.uint8)
    P = nx * ny
    dev = raw[: 144 * P].view(torch.int16).view(12, ny, nx, 6).permute(0, 3, 1, 2).reshape(72, ny, nx)
    rec = raw[144 * P: 192 * P].view(ny, nx, 48)
    side = rec[:, :, :32].contiguous().view(torch.float32).permute(2, 0, 1).contiguous()
    scale = rec[:, :, 32:44].contiguous().view(torch.float16).permute(2, 0, 1).contiguous()
    return dev.contiguous(), side, scale


class GuessNet:
    """The inversion-guess network: device weights plus training through the
    library's forward/backward/Adam kernels (rlbm_mlp_* in include/rlbm.h)."""

    def __init__(self, device="cuda", stream=None):
        self.stream = stream if stream is not None else torch.cuda.current_stream(device)
        self.w = torch.zeros(MLP_FLOATS, dtype=torch.float32, device=device)
        self._ws = None
        self._ws_n = 0

    def _workspace(self, n):
        if self._ws is None or self._ws_n < n:
            nbytes = lib().rlbm_mlp_workspace_bytes(int(n))
            self._ws = torch.empty(int(nbytes) // 4 + 1, dtype=torch.float32, device=self.w.device)
            self._ws_n = n
        return self._ws

    def _s(self):
        return ctypes.c_void_p(self.stream.cuda_stream)

    def init(self, x, t, noise):
        x, t, noise = (v.contiguous().float() for v in (x.reshape(-1), t.reshape(-1), noise.reshape(-1)))
        assert noise.numel() >= MLP_HIDDEN + 1
        _check(lib().rlbm_mlp_init(_ptr(self.w), _ptr(x), _ptr(t), x.numel(), _ptr(noise),
                                   _ptr(self._workspace(x.numel())), self._s()), "rlbm_mlp_init")

    def loss_grad(self, x, t):
        x, t = x.reshape(-1).contiguous().float(), t.reshape(-1).contiguous().float()
        grad = torch.empty(MLP_NTRAIN, dtype=torch.float32, device=self.w.device)
        loss = torch.empty(1, dtype=torch.float32, device=self.w.device)
        _check(lib().rlbm_mlp_loss_grad(_ptr(self.w), _ptr(x), _ptr(t), x.numel(), _ptr(grad), _ptr(loss),
                                        _ptr(self._workspace(x.numel())), self._s()), "rlbm_mlp_loss_grad")
        return loss, grad

    def train(self, x, t, iters, lr):
        x, t = x.reshape(-1).contiguous().float(), t.reshape(-1).contiguous().float()
        losses = torch.empty(max(int(iters), 1), dtype=torch.float32, device=self.w.device)
        _check(lib().rlbm_mlp_train(_ptr(self.w), _ptr(x), _ptr(t), x.numel(), int(iters), float(lr), _ptr(losses),
                                    _ptr(self._workspace(x.numel())), self._s()), "rlbm_mlp_train")
        return losses[:iters]

    def train_noalloc(self, x, t, iters, lr):
        """As train, through the allocation-free entry point (at most MLP_NOALLOC_MAX
        samples; the library's own device array replaces the workspace)."""
        x, t = x.reshape(-1).contiguous().float(), t.reshape(-1).contiguous().float()
        losses = torch.empty(max(int(iters), 1), dtype=torch.float32, device=self.w.device)
        _check(lib().rlbm_mlp_train_noalloc(_ptr(self.w), _ptr(x), _ptr(t), x.numel(), int(iters), float(lr),
                                            _ptr(losses), self._s()), "rlbm_mlp_train_noalloc")
        return losses[:iters]

    def predict(self, x):
        x = x.reshape(-1).contiguous().float()
        y = torch.empty_like(x)
        _check(lib().rlbm_mlp_predict(_ptr(self.w), _ptr(x), _ptr(y), x.numel(), self._s()), "rlbm_mlp_predict")
        return y


class Batch:
    """Many grids of uneven sizes advanced by one launch per step (rlbm_init_batch).

    params_list / init_list: one params dict and init-field dict per grid (as for Sim);
    statistic, precision, guess and tile must agree across grids."""

    def __init__(self, params_list, init_list, device="cuda", stream=None):
        self.stream = stream if stream is not None else torch.cuda.current_stream(device)
        args = [_grid_args(p, i, device, self.stream) for p, i in zip(params_list, init_list)]
        self.params = [dict(p) for p in params_list]
        self.f = [a[0] for a in args]
        self._keep = [a[3] for a in args]
        n = len(args)
        self._p = (Params * n)(*[a[1] for a in args])
        self._fi = (InitFields * n)(*[a[2] for a in args])
        ctx = ctypes.c_void_p()
        _check(lib().rlbm_init_batch(ctypes.byref(ctx), n, self._p, self._fi), "rlbm_init_batch")
        self.ctx = ctx

    def __len__(self):
        return len(self.f)

    def step(self, nsteps=1):
        _check(lib().rlbm_step(self.ctx, int(nsteps)), "rlbm_step")

    def capture(self):
        """Capture the replayed step graphs now (no step is run)."""
        _check(lib().rlbm_capture(self.ctx), "rlbm_capture")

    def autotune(self, trial_steps=5):
        tx, ty = ctypes.c_int32(), ctypes.c_int32()
        _check(lib().rlbm_autotune(self.ctx, int(trial_steps), ctypes.byref(tx), ctypes.byref(ty)), "rlbm_autotune")
        return tx.value, ty.value

    def configure(self, tile_x, tile_y, persistent=0):
        _check(lib().rlbm_configure(self.ctx, int(tile_x), int(tile_y), int(persistent)), "rlbm_configure")

    def state(self, g):
        return self.f[g][lib().rlbm_state_index(self.ctx)]

    @property
    def steps_done(self):
        return lib().rlbm_steps_done(self.ctx)

    def fields(self, g, names=FIELD_NAMES, check=True):
        p = self.params[g]
        ny, nx = int(p["ny"]), int(p["nx"])
        out = {k: torch.empty((ny, nx), dtype=torch.float64, device=self.f[g][0].device) for k in names}
        of = OutFields(**{k: _ptr(out.get(k)) for k in FIELD_NAMES + MOMENT_NAMES})
        rc = lib().rlbm_moments_grid(self.ctx, int(g), ctypes.byref(of))
        if check:
            _check(rc, "rlbm_moments_grid")
        return out

    def noneq_tensors(self, g, check=True):
        p = self.params[g]
        ny, nx = int(p["ny"]), int(p["nx"])
        out = {r: torch.empty((ny, nx), dtype=torch.float64, device=self.f[g][0].device) for r in (2, 3, 4, 5)}
        rc = lib().rlbm_noneq_tensors(self.ctx, int(g), *(_ptr(out[r]) for r in (2, 3, 4, 5)))
        if check:
            _check(rc, "rlbm_noneq_tensors")
        return out

    def sync(self):
        _check(lib().rlbm_sync(self.ctx), "rlbm_sync")

    def status(self):
        return lib().rlbm_status(self.ctx)

    def close(self):
        if getattr(self, "ctx", None):
            lib().rlbm_free(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
