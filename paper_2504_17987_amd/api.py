"""Python front of libpiv: a plan object taking torch device tensors.

Only marshalling lives here (shapes, dtypes, pointers, the current HIP
stream); every step of the PIV path runs in the library's HIP kernels.
PyTorch provides device memory and streams.
"""
from __future__ import annotations

import ctypes as C
from typing import Dict, Optional

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
    """

    def __init__(self, width: int, height: int, *, max_batch: int = 1, dtype: str = "u8",
                 bit_depth: Optional[int] = None, win: int = 16, step: int = 8, radius: int = 4,
                 levels: int = 3, block: int = 0, radius_coarse: int = 6, radius_fine: int = 2,
                 median: bool = True, warp: str = "b", peak: str = "argmax",
                 uod_threshold: float = 2.0, uod_epsilon: float = 0.1, device="cuda",
                 workspace: bool = True):
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
        self.params = p
        h = C.c_void_p()
        L.check(L.lib().piv_plan(C.byref(p), C.byref(h)))
        self.handle = h
        nx, ny = C.c_int32(), C.c_int32()
        L.check(L.lib().piv_plan_grid(h, C.byref(nx), C.byref(ny)))
        self.nx, self.ny = nx.value, ny.value
        self.width, self.height, self.max_batch = width, height, max_batch
        self.device = torch.device(device)
        self.workspace = None
        self.slot_mask = None
        if workspace:
            self.bind_workspace(torch.empty(self.workspace_bytes(max_batch), dtype=torch.uint8,
                                            device=self.device))

    # -- plan management ---------------------------------------------------
    def workspace_bytes(self, batch: int) -> int:
        return int(L.lib().piv_plan_workspace_bytes(self.handle, batch))

    def bind_workspace(self, ws: Optional[torch.Tensor]) -> None:
        L.check(L.lib().piv_plan_bind_workspace(self.handle, _ptr(ws), 0 if ws is None else ws.numel()))
        self.workspace = ws

    def bind_slot_mask(self, mask: Optional[torch.Tensor]) -> None:
        if mask is not None:
            assert mask.dtype == torch.uint8 and mask.is_contiguous() and mask.numel() >= self.max_batch
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
    def _images(self, A: torch.Tensor, B: torch.Tensor):
        for t in (A, B):
            if t.dtype != self.tdtype or t.device.type != "cuda":
                raise TypeError(f"images must be {self.tdtype} device tensors")
            if t.dim() != 3 or t.shape[1:] != (self.height, self.width):
                raise ValueError(f"images must be [n, {self.height}, {self.width}]")
            if t.stride(2) != 1 or (t.shape[0] > 1 and t.stride(0) != self.height * t.stride(1)):
                raise ValueError("images must be [n][H][pitch] with unit column stride")
        if A.stride() != B.stride() or A.shape != B.shape:
            raise ValueError("A and B must have the same shape and strides")
        return A.shape[0], A.stride(1) * self.es

    def _field(self, n, like=None):
        return torch.empty((n, 2, self.ny, self.nx), dtype=torch.float32, device=self.device)

    def _vec(self, n, dtype=torch.float32):
        return torch.empty((n, self.ny, self.nx), dtype=dtype, device=self.device)

    # -- the path ------------------------------------------------------------
    def predict(self, A, B, pred=None):
        n, pitch = self._images(A, B)
        pred = self._field(n) if pred is None else pred
        L.check(L.lib().piv_predict(self.handle, _ptr(A), _ptr(B), pitch, n, _ptr(pred), _stream(self.device)))
        return pred

    def correct(self, A, B, pred=None, disp=None, peak=None, flags=None, want_peak=True):
        n, pitch = self._images(A, B)
        disp = self._field(n) if disp is None else disp
        if peak is None and want_peak:
            peak = self._vec(n)
        flags = self._vec(n, torch.uint8) if flags is None else flags
        L.check(L.lib().piv_correct(self.handle, _ptr(A), _ptr(B), pitch, n, _ptr(pred), _ptr(disp),
                                    _ptr(peak), _ptr(flags), _stream(self.device)))
        return disp, peak, flags

    def validate(self, field, flags=None):
        """In place on field [n][2][ny][nx] (and flags [n][ny][nx] if given)."""
        n = field.shape[0]
        L.check(L.lib().piv_validate(self.handle, _ptr(field), _ptr(flags), n, _stream(self.device)))
        return field, flags

    def vorticity(self, disp, omega=None):
        n = disp.shape[0]
        omega = self._vec(n) if omega is None else omega
        L.check(L.lib().piv_vorticity(self.handle, _ptr(disp), _ptr(omega), n, _stream(self.device)))
        return omega

    def run(self, A, B, out: Optional[Dict[str, torch.Tensor]] = None) -> Dict[str, torch.Tensor]:
        """predict -> validate(pred) -> correct -> validate -> vorticity."""
        n, pitch = self._images(A, B)
        if out is None:
            out = dict(pred=self._field(n), disp=self._field(n), peak=self._vec(n),
                       flags=self._vec(n, torch.uint8), omega=self._vec(n))
        L.check(L.lib().piv_run(self.handle, _ptr(A), _ptr(B), pitch, n, _ptr(out["pred"]),
                                _ptr(out["disp"]), _ptr(out.get("peak")), _ptr(out["flags"]),
                                _ptr(out["omega"]), _stream(self.device)))
        return out

    def ssd_forward(self, A, B, U, loss=None):
        n = A.shape[0]
        self._f32(A, B, U)
        loss = self._vec(n) if loss is None else loss
        L.check(L.lib().piv_ssd_forward(self.handle, _ptr(A), _ptr(B), _ptr(U), n, _ptr(loss),
                                        _stream(self.device)))
        return loss

    def ssd_backward(self, A, B, U, g_loss, g_U=None, gn_diag=None, want_diag=True):
        n = A.shape[0]
        self._f32(A, B, U, g_loss)
        g_U = self._field(n) if g_U is None else g_U
        if gn_diag is None and want_diag:
            gn_diag = self._field(n)
        L.check(L.lib().piv_ssd_backward(self.handle, _ptr(A), _ptr(B), _ptr(U), _ptr(g_loss), n,
                                         _ptr(g_U), _ptr(gn_diag), _stream(self.device)))
        return g_U, gn_diag

    def _f32(self, *ts):
        for t in ts:
            if t.dtype != torch.float32 or not t.is_contiguous() or t.device.type != "cuda":
                raise TypeError("SSD tensors must be contiguous float32 device tensors")
