"""Python front of libpiv: a plan object taking torch device tensors.

Only marshalling lives here (shapes, dtypes, pointers, the current HIP
stream); every step of the PIV path runs in the library's HIP kernels.
PyTorch provides device memory and streams.
"""
from __future__ import annotations

import ctypes as C
from typing import Dict, Optional, Tuple

import torch

from . import _lib as L

_DT = {"u8": (L.PIV_U8, torch.uint8, 1), "u16": (L.PIV_U16, torch.uint16, 2),
       "f32": (L.PIV_F32, torch.float32, 4)}


def _ptr(t: Optional[torch.Tensor]) -> Optional[int]:
    return None if t is None else t.data_ptr()


def _stream(device) -> int:
    return torch.cuda.current_stream(device).cuda_stream


class Plan:
    """A validated PIV configuration with its device workspace.

    Parameters follow ``piv_params`` (include/piv.h); defaults are the
    paper's 16 x 16 windows at 50% step-over with UOD threshold 2 and
    regulariser 0.1 px, a +-4 px correction search and a 3-level predictor.

    Every tensor argument is checked (dtype, shape, batch, device,
    contiguity) before the C ABI is called, so a wrong tensor raises here
    instead of letting a kernel read or write out of bounds.
    """

    def __init__(self, width: int, height: int, *, max_batch: int = 1, dtype: str = "u8",
                 bit_depth: Optional[int] = None, win: int = 16, step: int = 8, radius: int = 4,
                 levels: int = 3, block: int = 0, radius_coarse: int = 6, radius_fine: int = 2,
                 median: bool = True, warp: str = "b", peak: str = "argmax",
                 uod_threshold: float = 2.0, uod_epsilon: float = 0.1, sgm: bool = False,
                 sgm_p1: int = 2, sgm_p2: int = 16, device="cuda", workspace: bool = True):
        code, tdt, es = _DT[dtype]
        self.dtype, self.tdtype, self.es = dtype, tdt, es
        p = L.Params()
        L.lib().piv_params_default(C.byref(p))
        p.width, p.height, p.max_batch = width, height, max_batch
        p.dtype = code
        p.bit_depth = bit_depth or (8 if dtype == "u8" else 12 if dtype == "u16" else 32)
        p.win, p.step, p.radius = win, step, radius
        p.levels, p.block, p.radius_coarse, p.radius_fine = levels, block, radius_coarse, radius_fine
        p.median = int(bool(median))
        p.warp = {"b": L.PIV_WARP_B, "central": L.PIV_WARP_CENTRAL}[warp]
        p.peak = {"argmax": L.PIV_PEAK_ARGMAX, "fixed": L.PIV_PEAK_FIXED_CENTER}[peak]
        p.uod_threshold, p.uod_epsilon = uod_threshold, uod_epsilon
        p.sgm, p.sgm_p1, p.sgm_p2 = int(bool(sgm)), sgm_p1, sgm_p2
        self.params = p
        h = C.c_void_p()
        L.check(L.lib().piv_plan(C.byref(p), C.byref(h)))
        self.handle = h
        nx, ny = C.c_int32(), C.c_int32()
        L.check(L.lib().piv_plan_grid(h, C.byref(nx), C.byref(ny)))
        self.nx, self.ny = nx.value, ny.value
        self.width, self.height, self.max_batch = width, height, max_batch
        dev = torch.device(device)
        if dev.type == "cuda" and dev.index is None and torch.cuda.is_available():
            dev = torch.device("cuda", torch.cuda.current_device())
        self.device = dev
        self.workspace = None
        self.slot_mask = None
        if workspace:
            self.bind_workspace(torch.empty(self.workspace_bytes(max_batch), dtype=torch.uint8,
                                            device=self.device))

    # -- plan management ---------------------------------------------------
    def workspace_bytes(self, batch: int) -> int:
        return int(L.lib().piv_plan_workspace_bytes(self.handle, batch))

    def bind_workspace(self, ws: Optional[torch.Tensor]) -> None:
        """Bind a uint8 device tensor as the plan's workspace (None unbinds).
        The library prepares it (zeroes the pyramid margins) on the current
        stream; this waits for that, so the plan is ready on any stream when
        it returns (binding is set-up work, not on the hot path)."""
        if ws is not None:
            self._dev(ws, "workspace")
            if ws.dtype != torch.uint8 or not ws.is_contiguous():
                raise TypeError("workspace must be a contiguous uint8 tensor")
        L.check(L.lib().piv_plan_bind_workspace(self.handle, _ptr(ws), 0 if ws is None else ws.numel(),
                                                None if ws is None else _stream(self.device)))
        if ws is not None:
            torch.cuda.current_stream(self.device).synchronize()
        self.workspace = ws

    def bind_slot_mask(self, mask: Optional[torch.Tensor]) -> None:
        if mask is not None:
            self._tensor(mask, "slot mask", torch.uint8, (), self.max_batch)
            self._devices(mask=mask)
        L.check(L.lib().piv_plan_bind_slot_mask(self.handle, _ptr(mask)))
        self.slot_mask = mask

    def correct_impl(self) -> int:
        """0: generic per-window kernel, 1: cell-shared tiled kernel."""
        return L.lib().piv_debug_correct_impl(self.handle)

    def close(self) -> None:
        if getattr(self, "handle", None):
            L.lib().piv_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- argument checks ---------------------------------------------------
    def _dev(self, t: torch.Tensor, name: str) -> None:
        if t.device.type != "cuda" or (self.device.index is not None and t.device.index != self.device.index):
            raise TypeError(f"{name} must be on the plan's device {self.device}, not {t.device}")

    def _tensor(self, t, name: str, dtype, tail: Tuple[int, ...], n: int, exact: bool = False) -> None:
        """t must be a contiguous `dtype` tensor of shape [>= n, *tail] (== n if
        exact) on the plan's device."""
        if not isinstance(t, torch.Tensor):
            raise TypeError(f"{name} must be a torch tensor")
        if t.dtype != dtype:
            raise TypeError(f"{name} must be {dtype}, not {t.dtype}")
        if t.dim() != len(tail) + 1 or tuple(t.shape[1:]) != tuple(tail):
            raise ValueError(f"{name} must have shape [n, {', '.join(map(str, tail))}], not {list(t.shape)}")
        if t.shape[0] < n or (exact and t.shape[0] != n):
            raise ValueError(f"{name} holds {t.shape[0]} pairs, the call needs {n}")
        if not t.is_contiguous():
            raise ValueError(f"{name} must be contiguous")

    def _devices(self, **named) -> None:
        """Checked last, after every dtype and shape check: the tensors live
        on the plan's device."""
        for name, t in named.items():
            if t is not None:
                self._dev(t, name)

    def _batch(self, n: int) -> None:
        if n > self.max_batch:
            raise ValueError(f"batch {n} exceeds the plan's max_batch {self.max_batch}")

    def _images(self, A: torch.Tensor, B: torch.Tensor):
        for t in (A, B):
            if not isinstance(t, torch.Tensor) or t.dtype != self.tdtype:
                raise TypeError(f"images must be {self.tdtype} tensors")
            if t.dim() != 3 or tuple(t.shape[1:]) != (self.height, self.width):
                raise ValueError(f"images must be [n, {self.height}, {self.width}]")
            if t.stride(2) != 1 or (t.shape[0] > 1 and t.stride(0) != self.height * t.stride(1)):
                raise ValueError("images must be [n][H][pitch] with unit column stride")
        if A.stride() != B.stride() or A.shape != B.shape:
            raise ValueError("A and B must have the same shape and strides")
        self._batch(A.shape[0])
        return A.shape[0], A.stride(1) * self.es

    def _fieldT(self, t, name, n):
        self._tensor(t, name, torch.float32, (2, self.ny, self.nx), n)

    def _vecT(self, t, name, n, dtype=torch.float32):
        self._tensor(t, name, dtype, (self.ny, self.nx), n)

    def _field(self, n, like=None):
        return torch.empty((n, 2, self.ny, self.nx), dtype=torch.float32, device=self.device)

    def _vec(self, n, dtype=torch.float32):
        return torch.empty((n, self.ny, self.nx), dtype=dtype, device=self.device)

    def _outputs(self, n, out: Dict[str, torch.Tensor]) -> None:
        for k in ("pred", "disp", "flags", "omega"):
            if k not in out or out[k] is None:
                raise ValueError(f"out must hold '{k}'")
        self._fieldT(out["pred"], "pred", n)
        self._fieldT(out["disp"], "disp", n)
        self._vecT(out["flags"], "flags", n, torch.uint8)
        self._vecT(out["omega"], "omega", n)
        if out.get("peak") is not None:
            self._vecT(out["peak"], "peak", n)

    def _out_devices(self, out) -> None:
        self._devices(**{k: out.get(k) for k in ("pred", "disp", "peak", "flags", "omega")})

    # -- the path ------------------------------------------------------------
    def predict(self, A, B, pred=None):
        n, pitch = self._images(A, B)
        pred = self._field(n) if pred is None else pred
        self._fieldT(pred, "pred", n)
        self._devices(A=A, B=B, pred=pred)
        L.check(L.lib().piv_predict(self.handle, _ptr(A), _ptr(B), pitch, n, _ptr(pred), _stream(self.device)))
        return pred

    def correct(self, A, B, pred=None, disp=None, peak=None, flags=None, want_peak=True):
        n, pitch = self._images(A, B)
        if pred is not None:
            self._fieldT(pred, "pred", n)
        disp = self._field(n) if disp is None else disp
        self._fieldT(disp, "disp", n)
        if peak is None and want_peak:
            peak = self._vec(n)
        if peak is not None:
            self._vecT(peak, "peak", n)
        flags = self._vec(n, torch.uint8) if flags is None else flags
        self._vecT(flags, "flags", n, torch.uint8)
        self._devices(A=A, B=B, pred=pred, disp=disp, peak=peak, flags=flags)
        L.check(L.lib().piv_correct(self.handle, _ptr(A), _ptr(B), pitch, n, _ptr(pred), _ptr(disp),
                                    _ptr(peak), _ptr(flags), _stream(self.device)))
        return disp, peak, flags

    def validate(self, field, flags=None):
        """In place on field [n][2][ny][nx] (and flags [n][ny][nx] if given)."""
        self._fieldT(field, "field", 0)
        n = field.shape[0]
        self._batch(n)
        if flags is not None:
            self._vecT(flags, "flags", n, torch.uint8)
        self._devices(field=field, flags=flags)
        L.check(L.lib().piv_validate(self.handle, _ptr(field), _ptr(flags), n, _stream(self.device)))
        return field, flags

    def vorticity(self, disp, omega=None):
        self._fieldT(disp, "disp", 0)
        n = disp.shape[0]
        self._batch(n)
        omega = self._vec(n) if omega is None else omega
        self._vecT(omega, "omega", n)
        self._devices(disp=disp, omega=omega)
        L.check(L.lib().piv_vorticity(self.handle, _ptr(disp), _ptr(omega), n, _stream(self.device)))
        return omega

    def run(self, A, B, out: Optional[Dict[str, torch.Tensor]] = None) -> Dict[str, torch.Tensor]:
        """predict -> validate(pred) -> correct -> validate -> vorticity."""
        n, pitch = self._images(A, B)
        if out is None:
            out = self._new_outputs(n)
        self._outputs(n, out)
        self._devices(A=A, B=B)
        self._out_devices(out)
        L.check(L.lib().piv_run(self.handle, _ptr(A), _ptr(B), pitch, n, _ptr(out["pred"]),
                                _ptr(out["disp"]), _ptr(out.get("peak")), _ptr(out["flags"]),
                                _ptr(out["omega"]), _stream(self.device)))
        return out

    def run_noalloc(self, A, B, out: Dict[str, torch.Tensor]) -> Dict[str, torch.Tensor]:
        """piv_run on the library's fixed device scratch array instead of the
        plan's workspace (which may be absent): allocates nothing, so every
        output must be passed in `out` (pred, disp, flags, omega; peak
        optional).  Calls that overlap on one GPU share the array and race."""
        n, pitch = self._images(A, B)
        self._outputs(n, out)
        self._devices(A=A, B=B)
        self._out_devices(out)
        L.check(L.lib().piv_run_noalloc(self.handle, _ptr(A), _ptr(B), pitch, n, _ptr(out["pred"]),
                                        _ptr(out["disp"]), _ptr(out.get("peak")), _ptr(out["flags"]),
                                        _ptr(out["omega"]), _stream(self.device)))
        return out

    def _new_outputs(self, n):
        return dict(pred=self._field(n), disp=self._field(n), peak=self._vec(n),
                    flags=self._vec(n, torch.uint8), omega=self._vec(n))

    # -- pre-processing -------------------------------------------------------
    def _frames(self, inp, out):
        """inp [n][H][W] frames of the plan's dtype; out the same shape (new
        when None)."""
        if out is None:
            out = torch.empty_like(inp)
        n, pitch = self._images(inp, out)
        self._devices(inp=inp, out=out)
        return n, pitch, out

    def highpass(self, inp, out=None, radius: int = 7):
        """Background removal: max(0, I - floor(box mean)) over the image
        part of the (2 radius + 1)^2 box; out must not alias inp."""
        n, pitch, out = self._frames(inp, out)
        L.check(L.lib().piv_highpass(self.handle, _ptr(inp), _ptr(out), pitch, n, int(radius),
                                     _stream(self.device)))
        return out

    def clahe_lut_bytes(self, n: int, tiles_x: int, tiles_y: int) -> int:
        return int(L.lib().piv_clahe_lut_bytes(self.handle, n, tiles_x, tiles_y))

    def clahe(self, inp, out=None, tiles=(8, 8), clip_factor: float = 2.0, lut=None):
        """Contrast-limited adaptive histogram equalisation on a tiles[0] x
        tiles[1] grid (out may be inp); lut: optional uint8 device scratch of
        clahe_lut_bytes(n, *tiles) bytes, left holding the tile mappings."""
        n, pitch, out = self._frames(inp, out)
        need = self.clahe_lut_bytes(n, tiles[0], tiles[1])
        if lut is None:
            lut = torch.empty(max(need, 4), dtype=torch.uint8, device=self.device)
        if lut.dtype != torch.uint8 or not lut.is_contiguous() or lut.numel() < need:
            raise ValueError(f"lut must be a contiguous uint8 tensor of at least {need} bytes")
        self._devices(lut=lut)
        L.check(L.lib().piv_clahe(self.handle, _ptr(inp), _ptr(out), pitch, n, int(tiles[0]), int(tiles[1]),
                                  float(clip_factor), _ptr(lut), lut.numel(), _stream(self.device)))
        return out

    # -- temporal smoothing ----------------------------------------------------
    def new_state(self, nstate: int) -> torch.Tensor:
        """Zeroed smoothing state for `nstate` streams, [nstate][2][ny][nx]."""
        return torch.zeros((nstate, 2, self.ny, self.nx), dtype=torch.float32, device=self.device)

    def _slots(self, slot, n, state):
        self._tensor(slot, "slot", torch.int32, (), n)
        if state is not None:
            self._tensor(state, "state", torch.float32, (2, self.ny, self.nx), 1)

    def smooth(self, field, state, slot, alpha: float = 0.5):
        """Exponential smoothing in time, in place on field [n][2][ny][nx]
        with state [nstate][2][ny][nx] and slot int32 [n] (k continues state
        k, -1-k starts it)."""
        self._fieldT(field, "field", 0)
        n = field.shape[0]
        self._batch(n)
        if state is None:
            raise ValueError("state must not be None")
        self._slots(slot, n, state)
        self._devices(field=field, state=state, slot=slot)
        L.check(L.lib().piv_smooth(self.handle, _ptr(field), _ptr(state), _ptr(slot), state.shape[0],
                                   float(alpha), n, _stream(self.device)))
        return field

    def run_temporal(self, A, B, slot, state_pred=None, state_disp=None, alpha1: float = 0.5,
                     alpha2: float = 0.5, out: Optional[Dict[str, torch.Tensor]] = None):
        """The path with the paper's exponential smoothing of the validated
        predictor (alpha1, state_pred) and of the final field (alpha2,
        state_disp); both states [nstate][2][ny][nx], slot int32 [n]."""
        n, pitch = self._images(A, B)
        if out is None:
            out = self._new_outputs(n)
        self._outputs(n, out)
        nstate = None
        for st in (state_pred, state_disp):
            self._slots(slot, n, st)
            if st is not None:
                if nstate is not None and st.shape[0] != nstate:
                    raise ValueError("state_pred and state_disp must hold the same number of streams")
                nstate = st.shape[0]
        self._devices(A=A, B=B, slot=slot, state_pred=state_pred, state_disp=state_disp)
        self._out_devices(out)
        L.check(L.lib().piv_run_temporal(self.handle, _ptr(A), _ptr(B), pitch, n, _ptr(slot), nstate or 1,
                                         _ptr(state_pred), _ptr(state_disp), float(alpha1), float(alpha2),
                                         _ptr(out["pred"]), _ptr(out["disp"]), _ptr(out.get("peak")),
                                         _ptr(out["flags"]), _ptr(out["omega"]), _stream(self.device)))
        return out

    # -- differentiable SSD (addition) ------------------------------------------
    def _ssd_inputs(self, A, B, U):
        for t, nm in ((A, "A"), (B, "B")):
            self._tensor(t, nm, torch.float32, (self.height, self.width), 0)
        n = A.shape[0]
        if B.shape[0] != n:
            raise ValueError("A and B must hold the same number of pairs")
        self._batch(n)
        self._fieldT(U, "U", n)
        return n

    def ssd_forward(self, A, B, U, loss=None):
        n = self._ssd_inputs(A, B, U)
        loss = self._vec(n) if loss is None else loss
        self._vecT(loss, "loss", n)
        self._devices(A=A, B=B, U=U, loss=loss)
        L.check(L.lib().piv_ssd_forward(self.handle, _ptr(A), _ptr(B), _ptr(U), n, _ptr(loss),
                                        _stream(self.device)))
        return loss

    def ssd_backward(self, A, B, U, g_loss, g_U=None, gn_diag=None, want_diag=True):
        n = self._ssd_inputs(A, B, U)
        self._vecT(g_loss, "g_loss", n)
        g_U = self._field(n) if g_U is None else g_U
        self._fieldT(g_U, "g_U", n)
        if gn_diag is None and want_diag:
            gn_diag = self._field(n)
        if gn_diag is not None:
            self._fieldT(gn_diag, "gn_diag", n)
        self._devices(A=A, B=B, U=U, g_loss=g_loss, g_U=g_U, gn_diag=gn_diag)
        L.check(L.lib().piv_ssd_backward(self.handle, _ptr(A), _ptr(B), _ptr(U), _ptr(g_loss), n,
                                         _ptr(g_U), _ptr(gn_diag), _stream(self.device)))
        return g_U, gn_diag

    def ssd_refine(self, A, B, U, steps: int = 10, tau: float = 4.0 / 9.0, lam_rel: float = 1e-3,
                   hist=None):
        """`steps` preconditioned gradient steps on the total windowed SSD,
        in place on U [n][2][ny][nx]; hist (optional) [n][steps + 1] float32
        receives the total loss before each step and after the last."""
        n = self._ssd_inputs(A, B, U)
        if hist is not None:
            self._tensor(hist, "hist", torch.float32, (steps + 1,), n)
        self._devices(A=A, B=B, U=U, hist=hist)
        L.check(L.lib().piv_ssd_refine(self.handle, _ptr(A), _ptr(B), _ptr(U), n, int(steps), float(tau),
                                       float(lam_rel), _ptr(hist), _stream(self.device)))
        return U, hist
