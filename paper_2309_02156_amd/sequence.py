"""Python front end over the C-ABI: device CSR matrices and sequences.

PyTorch supplies device memory and the current stream only; every step of the
method runs in the library's HIP kernels.
"""

from __future__ import annotations

import ctypes
from typing import Optional

import numpy as np
import torch

from . import native as nv

_SKETCH = {"gaussian": nv.SA_SKETCH_GAUSSIAN, "srht": nv.SA_SKETCH_SRHT}
_SOLVER = {"cg": nv.SA_CG, "gmres": nv.SA_GMRES}
_PREC = {"fp64": nv.SA_FP64, "mixed": nv.SA_MIXED, "mixed_krylov": nv.SA_MIXED_KRYLOV}
_PROJ = {"galerkin": nv.SA_GALERKIN, "minres": nv.SA_MINRES}
_BASIS = {"sketched_qr": nv.SA_BASIS_SKETCHED_QR, "pod": nv.SA_BASIS_POD}
_PRECOND = {"none": nv.SA_PRECOND_NONE, "jacobi": nv.SA_PRECOND_JACOBI}
_GUESS = {"projection": nv.SA_GUESS_PROJECTION, "zero": nv.SA_GUESS_ZERO,
          "previous": nv.SA_GUESS_PREVIOUS}


def _stream(stream=None) -> int:
    s = stream if stream is not None else torch.cuda.current_stream()
    return s.cuda_stream


def _ptr(t: torch.Tensor) -> int:
    if not t.is_cuda or not t.is_contiguous():
        raise ValueError("expected a contiguous device tensor")
    return t.data_ptr()


class DeviceCSR:
    """CSR matrix resident in device memory (int32 indices, float64 or float32 values)."""

    def __init__(self, rowptr, col, val, device="cuda"):
        self.rowptr = torch.as_tensor(np.asarray(rowptr, dtype=np.int32)).to(device)
        self.col = torch.as_tensor(np.asarray(col, dtype=np.int32)).to(device)
        v = np.asarray(val)
        if v.dtype not in (np.float64, np.float32):
            v = v.astype(np.float64)
        self.val = torch.as_tensor(v).to(device)
        self.n = int(self.rowptr.numel() - 1)
        self.nnz = int(self.col.numel())

    @classmethod
    def from_csr(cls, A, device="cuda"):
        return cls(A.rowptr, A.col, A.val, device)

    def set_values(self, val):
        """Overwrite the values in place (same pattern), e.g. for the next time step."""
        v = torch.as_tensor(np.ascontiguousarray(val))
        if v.numel() != self.nnz:
            raise ValueError("value count does not match the pattern")
        self.val.copy_(v.to(self.val.dtype))

    def c_struct(self) -> nv.SaCsr:
        return nv.SaCsr(self.n, self.nnz, _ptr(self.rowptr), _ptr(self.col), _ptr(self.val),
                        1 if self.val.dtype == torch.float32 else 0, 0)


def spmv(A: DeviceCSR, x: torch.Tensor, y: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
    """y = A x through sa_spmv."""
    if y is None:
        y = torch.empty_like(x)
    s = A.c_struct()
    nv.check(nv.lib().sa_spmv(ctypes.byref(s), _ptr(x), _ptr(y), _stream(stream)), "sa_spmv")
    return y


def solver_config(n: int, solver: str = "cg", restart: int = 30, tol: float = 1e-8, maxit: int = 200000,
                  poll: int = 0, precond: str = "none") -> nv.SaConfig:
    """The configuration of a plain FP64 Krylov solve of size n (history fields at their
    smallest valid values: no initial guess is formed)."""
    return nv.SaConfig(n=n, M=1, s=1, sketch=nv.SA_SKETCH_GAUSSIAN, projection=nv.SA_GALERKIN,
                       solver=_SOLVER[solver], restart=restart, tol=tol, maxit=maxit, precision=nv.SA_FP64,
                       inner_tol=1e-4, max_refine=1, guess=nv.SA_GUESS_ZERO, rank_tol_sketch=0.0,
                       rank_tol_chol=0.0, seed=0, poll=poll, inner_maxit=0, m=0, refresh=0,
                       basis=nv.SA_BASIS_SKETCHED_QR, precond=_PRECOND[precond])


def solve_static(A: DeviceCSR, b: torch.Tensor, x: torch.Tensor, solver: str = "cg", restart: int = 30,
                 tol: float = 1e-8, maxit: int = 200000, poll: int = 0, stream=None,
                 allow=(nv.SA_OK, nv.SA_NOTCONV, nv.SA_EBREAKDOWN), precond: str = "none"):
    """Krylov solve of A x = b from the iterate in x through sa_solve_static (no device
    allocation by the library); returns (x, info)."""
    cfg = solver_config(A.n, solver, restart, tol, maxit, poll, precond)
    inf = nv.SaInfo()
    s = A.c_struct()
    rc = nv.lib().sa_solve_static(ctypes.byref(cfg), ctypes.byref(s), _ptr(b), _ptr(x), ctypes.byref(inf),
                                  _stream(stream))
    nv.check(rc, "sa_solve_static", allow)
    d = inf.as_dict()
    d["rc"] = rc
    return x, d


class Sequence:
    """One sequence of systems A(t_i) x = b(t_i) handled by the library."""

    def __init__(self, n: int, M: int, s: Optional[int] = None, sketch: str = "gaussian",
                 solver: str = "cg", restart: int = 30, tol: float = 1e-8, maxit: int = 200000,
                 precision: str = "fp64", projection: str = "galerkin", guess: str = "projection",
                 seed: int = 0, rank_tol_sketch: float = 0.0, rank_tol_chol: float = 0.0,
                 inner_tol: float = 1e-4, max_refine: int = 10, inner_maxit: int = 0, poll: int = 0,
                 m: int = 0, refresh: int = 0, basis: str = "sketched_qr", precond: str = "none",
                 device="cuda", stream=None):
        self.n, self.M = n, M
        self.s = 2 * M if s is None else s
        self.precision = precision
        self.cfg = nv.SaConfig(
            n=n, M=M, s=self.s, sketch=_SKETCH[sketch], projection=_PROJ[projection],
            solver=_SOLVER[solver], restart=restart, tol=tol, maxit=maxit,
            precision=_PREC[precision], inner_tol=inner_tol, max_refine=max_refine,
            guess=_GUESS[guess], rank_tol_sketch=rank_tol_sketch, rank_tol_chol=rank_tol_chol,
            seed=seed, poll=poll, inner_maxit=inner_maxit, m=m, refresh=refresh, basis=_BASIS[basis],
            precond=_PRECOND[precond])
        L = nv.lib()
        nbytes = ctypes.c_size_t(0)
        nv.check(L.sa_workspace_bytes(ctypes.byref(self.cfg), ctypes.byref(nbytes)), "sa_workspace_bytes")
        self.workspace = torch.empty(int(nbytes.value), dtype=torch.uint8, device=device)
        self.stream = stream
        h = ctypes.c_void_p(0)
        nv.check(L.sa_init_sequence(ctypes.byref(self.cfg), _ptr(self.workspace), nbytes,
                                    _stream(stream), ctypes.byref(h)), "sa_init_sequence")
        self._h = h

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            nv.lib().sa_destroy_sequence(self._h)
            self._h = ctypes.c_void_p(0)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ------------------------------------------------------------------ steps
    def push(self, x: torch.Tensor):
        nv.check(nv.lib().sa_push_solution(self._h, _ptr(x), _stream(self.stream)), "sa_push_solution")

    def initial_guess(self, A: DeviceCSR, b: torch.Tensor, x0: Optional[torch.Tensor] = None,
                      info: bool = True):
        if x0 is None:
            x0 = torch.empty_like(b)
        inf = nv.SaInfo()
        s = A.c_struct()
        nv.check(nv.lib().sa_initial_guess(self._h, ctypes.byref(s), _ptr(b), _ptr(x0),
                                           ctypes.byref(inf) if info else None,
                                           _stream(self.stream)), "sa_initial_guess")
        return x0, (inf.as_dict() if info else None)

    def solve(self, A: DeviceCSR, b: torch.Tensor, x: torch.Tensor, info: bool = True,
              allow=(nv.SA_OK, nv.SA_NOTCONV, nv.SA_EBREAKDOWN)):
        inf = nv.SaInfo()
        s = A.c_struct()
        rc = nv.lib().sa_solve(self._h, ctypes.byref(s), _ptr(b), _ptr(x),
                               ctypes.byref(inf) if info else None, _stream(self.stream))
        nv.check(rc, "sa_solve", allow)
        d = inf.as_dict() if info else {}
        d["rc"] = rc
        return x, d

    def step(self, A: DeviceCSR, b: torch.Tensor, x: Optional[torch.Tensor] = None, info: bool = True,
             allow=(nv.SA_OK, nv.SA_NOTCONV, nv.SA_EBREAKDOWN)):
        """initial guess -> solve -> push in one library call (sa_step); returns (x, info)."""
        if x is None:
            x = torch.empty_like(b)
        inf = nv.SaInfo()
        s = A.c_struct()
        rc = nv.lib().sa_step(self._h, ctypes.byref(s), _ptr(b), _ptr(x), ctypes.byref(inf) if info else None,
                              _stream(self.stream))
        nv.check(rc, "sa_step", allow)
        d = inf.as_dict() if info else {}
        d["rc"] = rc
        return x, d

    # ------------------------------------------------------------------ learned guess
    def learned_attach(self, mlp: "MLP", n_hist: int = 8):
        """Use the predictor for the initial guesses from now on (fresh sequence)."""
        nv.check(nv.lib().sa_learned_attach(self._h, mlp._h if mlp is not None else None, n_hist),
                 "sa_learned_attach")
        self._mlp = mlp

    def set_time(self, t: float):
        nv.check(nv.lib().sa_set_time(self._h, float(t)), "sa_set_time")

    def last_target(self) -> np.ndarray:
        """The learned target written by the last push (M coefficients, lag order)."""
        return self.copy_state("target")

    # ------------------------------------------------------------------ checkpoint
    def export_state(self) -> bytes:
        """The sequence's carried state (history, sketch, sketched QR) as bytes."""
        L = nv.lib()
        nb = ctypes.c_size_t(0)
        nv.check(L.sa_state_bytes(self._h, ctypes.byref(nb)), "sa_state_bytes")
        buf = ctypes.create_string_buffer(nb.value)
        nv.check(L.sa_export_state(self._h, buf, nb.value, _stream(self.stream)), "sa_export_state")
        return buf.raw

    def import_state(self, image: bytes):
        """Resume from export_state's bytes (a fresh sequence of the same configuration)."""
        buf = ctypes.create_string_buffer(image, len(image))
        nv.check(nv.lib().sa_import_state(self._h, buf, len(image), _stream(self.stream)), "sa_import_state")

    # ------------------------------------------------------------------ inspection
    def profile_enable(self, enable: bool = True):
        """Time the dominant Krylov kernels of later solves (HIP events per launch)."""
        nv.check(nv.lib().sa_profile_enable(self._h, 1 if enable else 0), "sa_profile_enable")

    def profile_read(self) -> list:
        """[{name, launches, ms, bytes}] for the kernels timed since profile_enable."""
        L = nv.lib()
        cnt = ctypes.c_int32(0)
        nv.check(L.sa_profile_read(self._h, None, 0, ctypes.byref(cnt)), "sa_profile_read")
        arr = (nv.SaKernelProf * max(cnt.value, 1))()
        nv.check(L.sa_profile_read(self._h, arr, cnt.value, ctypes.byref(cnt)), "sa_profile_read")
        return [dict(name=r.name.decode(), launches=int(r.launches), ms=float(r.ms), bytes=float(r.bytes))
                for r in arr[:cnt.value]]

    def copy_state(self, what: str) -> np.ndarray:
        L = nv.lib()
        if what == "SX":
            out = np.empty((self.M, self.s), dtype=np.float64)
            code = 0
        elif what == "X":   # float32 storage in the mixed mode
            out = np.empty((self.M, self.n), dtype=np.float32 if self.precision == "mixed" else np.float64)
            code = 1
        elif what == "cX":
            out = np.empty(self.M, dtype=np.float64)
            code = 2
        elif what == "order":
            out = np.empty(self.M, dtype=np.int32)
            code = 3
        elif what == "target":
            out = np.empty(self.M, dtype=np.float64)
            code = 4
        else:
            raise ValueError(what)
        nv.check(L.sa_copy_state(self._h, code, out.ctypes.data, out.nbytes, _stream(self.stream)),
                 "sa_copy_state")
        if what in ("SX", "X"):
            return out.T.copy()   # column-major on the device -> (rows, M)
        return out


class MLP:
    """The coefficient-predictor MLP on the device (sa_mlp_*)."""

    def __init__(self, sizes, params, max_batch: int = 256, lr: float = 1e-3, beta1: float = 0.9,
                 beta2: float = 0.999, eps: float = 1e-8):
        """sizes = [n_in, hidden, ..., hidden, n_out]; params = [(W_l, b_l)] (float32)."""
        hidden = sizes[1:-1]
        if len(set(hidden)) > 1:
            raise ValueError("all hidden layers have one width")
        self.sizes = list(sizes)
        self.cfg = nv.SaMlpConfig(n_in=sizes[0], n_hidden=hidden[0] if hidden else sizes[-1],
                                  n_layers=len(hidden), n_out=sizes[-1], max_batch=max_batch, lr=lr,
                                  beta1=beta1, beta2=beta2, eps=eps, reserved=0)
        flat = np.concatenate([np.concatenate([np.asarray(W, np.float32).ravel(), np.asarray(b, np.float32)])
                               for W, b in params]).astype(np.float32)
        self.n_params = flat.size
        h = ctypes.c_void_p(0)
        nv.check(nv.lib().sa_mlp_create(ctypes.byref(self.cfg), flat.ctypes.data_as(ctypes.POINTER(ctypes.c_float)),
                                        ctypes.byref(h)), "sa_mlp_create")
        self._h = h

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            nv.lib().sa_mlp_destroy(self._h)
            self._h = ctypes.c_void_p(0)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_scaling(self, mu_in, sd_in, mu_out, sd_out):
        arrs = [np.ascontiguousarray(a, dtype=np.float32) for a in (mu_in, sd_in, mu_out, sd_out)]
        fp = ctypes.POINTER(ctypes.c_float)
        nv.check(nv.lib().sa_mlp_set_scaling(self._h, *[a.ctypes.data_as(fp) for a in arrs]), "sa_mlp_set_scaling")

    def forward(self, x: torch.Tensor, stream=None) -> torch.Tensor:
        """Standardised outputs for raw float32 rows x (device)."""
        y = torch.empty(x.shape[0], self.sizes[-1], dtype=torch.float32, device=x.device)
        nv.check(nv.lib().sa_mlp_forward(self._h, _ptr(x), x.shape[0], _ptr(y), _stream(stream)), "sa_mlp_forward")
        return y

    def train_step(self, x: torch.Tensor, t: torch.Tensor, loss: Optional[torch.Tensor] = None, stream=None):
        nv.check(nv.lib().sa_mlp_train_step(self._h, _ptr(x), _ptr(t), x.shape[0],
                                            _ptr(loss) if loss is not None else None, _stream(stream)),
                 "sa_mlp_train_step")

    def get(self, what: str = "params") -> np.ndarray:
        code = {"params": 0, "grads": 1, "adam_m": 2, "adam_v": 3}[what]
        out = np.empty(self.n_params, dtype=np.float32)
        nv.check(nv.lib().sa_mlp_get(self._h, code, out.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), out.size,
                                     _stream(None)), "sa_mlp_get")
        return out

    def unflatten(self, flat: np.ndarray):
        """[(W_l, b_l)] views of a flat parameter (or gradient) vector."""
        out, o = [], 0
        for fin, fout in zip(self.sizes[:-1], self.sizes[1:]):
            W = flat[o:o + fin * fout].reshape(fout, fin)
            o += fin * fout
            b = flat[o:o + fout]
            o += fout
            out.append((W, b))
        return out


class Batch:
    """Many independent sequences stepped together (sa_batch_*)."""

    def __init__(self, seqs, max_streams: int = 4, tune_warmup: int = 0):
        self.seqs = list(seqs)
        arr = (ctypes.c_void_p * len(self.seqs))(*[s._h.value for s in self.seqs])
        h = ctypes.c_void_p(0)
        nv.check(nv.lib().sa_batch_create(arr, len(self.seqs), max_streams, tune_warmup, ctypes.byref(h)),
                 "sa_batch_create")
        self._h = h

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            nv.lib().sa_batch_destroy(self._h)
            self._h = ctypes.c_void_p(0)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def step(self, As, bs, xs):
        """One step of every sequence; As: DeviceCSR list, bs / xs: float64 device tensors
        (xs receive the solutions).  Returns the list of info dicts."""
        n = len(self.seqs)
        structs = [A.c_struct() for A in As]
        Aarr = (ctypes.c_void_p * n)(*[ctypes.addressof(s) for s in structs])
        barr = (ctypes.c_void_p * n)(*[_ptr(b) for b in bs])
        xarr = (ctypes.c_void_p * n)(*[_ptr(x) for x in xs])
        infos = (nv.SaInfo * n)()
        torch.cuda.synchronize()
        nv.check(nv.lib().sa_batch_step(self._h, Aarr, barr, xarr, infos), "sa_batch_step")
        return [i.as_dict() for i in infos]

    MODES = {"auto": 0, "streams": 1, "segmented": 2, "segmented_eager": 3}

    def set_mode(self, mode: str):
        """"auto" (tuned), "streams", "segmented" (graph replays) or "segmented_eager"."""
        nv.check(nv.lib().sa_batch_set_mode(self._h, self.MODES[mode]), "sa_batch_set_mode")

    def solve_stats(self):
        """(algorithmic bytes, ms) of the last step's segmented solve; zeros after a
        stream step."""
        b, ms = ctypes.c_double(), ctypes.c_double()
        nv.check(nv.lib().sa_batch_solve_stats(self._h, ctypes.byref(b), ctypes.byref(ms)), "sa_batch_solve_stats")
        return b.value, ms.value

    def plan(self):
        s, p, t, g = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        nv.check(nv.lib().sa_batch_plan(self._h, ctypes.byref(s), ctypes.byref(p), ctypes.byref(t), ctypes.byref(g)),
                 "sa_batch_plan")
        return dict(streams=s.value, poll=p.value, tuned=bool(t.value), segmented=bool(g.value),
                    item_rows=g.value)
