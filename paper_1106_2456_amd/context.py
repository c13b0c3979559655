"""Python face of libmde: argument marshalling only.

Every step of the evaluation runs in the HIP kernels behind the C ABI;
torch provides device memory (the workspace and output tensors) and the
stream the library enqueues on.
"""
from __future__ import annotations

import ctypes as C
from contextlib import contextmanager
from typing import Optional, Sequence

import numpy as np
import torch

from ._lib import (MDE_FP64, MDE_MIXED, MDE_MIXED_GEMM, MDE_MIXED_GEMM_KSUM64, MdeDesc, MdeError,
                   lib)

PRECISIONS = {"fp64": MDE_FP64, "mixed": MDE_MIXED, "mixed_gemm": MDE_MIXED_GEMM,
              "mixed_gemm_ksum64": MDE_MIXED_GEMM_KSUM64}


def _ptr(t) -> Optional[int]:
    if t is None:
        return None
    return t.data_ptr()


def _np_ptr(a: np.ndarray) -> int:
    return a.ctypes.data


def _check_dev(t: torch.Tensor, dtype, shape, name):
    if not isinstance(t, torch.Tensor) or t.device.type != "cuda":
        raise TypeError(f"{name}: expected a device tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name}: expected {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name}: must be contiguous")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name}: expected shape {tuple(shape)}, got {tuple(t.shape)}")


class Graph:
    """A captured sequence of library calls (HIP graph)."""

    def __init__(self, handle, stream):
        self._h = handle
        self._stream = stream

    def launch(self, stream=None):
        s = self._stream if stream is None else stream
        rc = lib().mde_graph_launch(self._h, C.c_void_p(s.cuda_stream))
        if rc:
            raise MdeError(rc, "graph launch failed")

    def __del__(self):
        try:
            if self._h:
                lib().mde_graph_destroy(self._h)
        except Exception:
            pass


class Context:
    """One multi-determinant wave function on one GPU.

    n_elec: (n_up, n_dn); n_orb: orbitals per spin (n + m)."""

    def __init__(self, n_elec: Sequence[int], n_orb: Sequence[int], max_walkers: int,
                 max_order: int = 4, refresh_every: Optional[int] = None,
                 precision: str = "fp64", device: str = "cuda:0",
                 stream: Optional[torch.cuda.Stream] = None):
        self.device = torch.device(device)
        self.n_elec = tuple(int(x) for x in n_elec)
        self.n_orb = tuple(int(x) for x in n_orb)
        self.max_walkers = int(max_walkers)
        self.precision = precision
        if refresh_every is None:
            refresh_every = self.n_elec[0] + self.n_elec[1]
        d = MdeDesc()
        d.n_elec[0], d.n_elec[1] = self.n_elec
        d.n_orb[0], d.n_orb[1] = self.n_orb
        d.max_walkers = self.max_walkers
        d.max_order = int(max_order)
        d.refresh_every = int(refresh_every)
        if precision not in PRECISIONS:
            raise ValueError(f"precision must be one of {sorted(PRECISIONS)}")
        d.precision = PRECISIONS[precision]
        with torch.cuda.device(self.device):
            self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        h = C.c_void_p()
        rc = lib().mde_create(C.byref(d), C.c_void_p(self.stream.cuda_stream), C.byref(h))
        if rc:
            raise MdeError(rc, "mde_create")
        self._h = h
        self._keep = []
        self.W = None
        self.workspace = None
        # bumped by every call that changes the library-side state, so that
        # a caller holding on to one state (the autograd Function between
        # its forward and backward) can tell whether it is still current
        self.state_seq = 0

    # -- plumbing ----------------------------------------------------------
    def _chk(self, rc, what):
        if rc:
            msg = lib().mde_error_string(self._h)
            raise MdeError(rc, f"{what}: {msg.decode() if msg else ''}")

    def __del__(self):
        try:
            if getattr(self, "_h", None):
                lib().mde_destroy(self._h)
                self._h = None
        except Exception:
            pass

    def _empty(self, shape, dtype=torch.float64):
        return torch.empty(shape, dtype=dtype, device=self.device)

    # -- setup -----------------------------------------------------------------
    def set_excitations(self, spin: int, offsets, holes, particles):
        off = np.ascontiguousarray(offsets, np.int32)
        h = np.ascontiguousarray(holes, np.int32)
        p = np.ascontiguousarray(particles, np.int32)
        self._chk(lib().mde_set_excitations(self._h, spin, off.shape[0] - 1, _np_ptr(off),
                                            _np_ptr(h), _np_ptr(p)), "set_excitations")

    def set_ci(self, coef, up_idx, dn_idx):
        c = np.ascontiguousarray(coef, np.float64)
        u = np.ascontiguousarray(up_idx, np.int32)
        d = np.ascontiguousarray(dn_idx, np.int32)
        self._chk(lib().mde_set_ci(self._h, c.shape[0], _np_ptr(c), _np_ptr(u), _np_ptr(d)),
                  "set_ci")
        self.n_det = int(c.shape[0])

    def set_reference(self, ref_up: int, ref_dn: int):
        """Switch the reference to the determinant (ref_up, ref_dn) of the
        caller's excitation lists (before bind)."""
        self._chk(lib().mde_set_reference(self._h, int(ref_up), int(ref_dn)), "set_reference")

    def set_basis(self, spin: int, centres, expo, mo):
        cc = np.ascontiguousarray(centres, np.float64)
        ee = np.ascontiguousarray(expo, np.float64)
        mm = np.ascontiguousarray(mo, np.float64)
        self._chk(lib().mde_sgauss_set_basis(self._h, spin, ee.shape[0], _np_ptr(cc), _np_ptr(ee),
                                             _np_ptr(mm)), "set_basis")

    def workspace_bytes(self, W: int) -> int:
        b = C.c_size_t()
        self._chk(lib().mde_workspace_bytes(self._h, W, C.byref(b)), "workspace_bytes")
        return int(b.value)

    def bind(self, W: int):
        nbytes = self.workspace_bytes(W)
        ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        off = (-ws.data_ptr()) % 256
        self.workspace = ws
        self._chk(lib().mde_bind_workspace(self._h, W, ws.data_ptr() + off, nbytes), "bind")
        self.W = int(W)

    # -- evaluation ----------------------------------------------------------------
    def init(self, orb_up: torch.Tensor, orb_dn: torch.Tensor, status=None):
        W = self.W
        _check_dev(orb_up, torch.float64, (W, self.n_elec[0], 5, self.n_orb[0]), "orb_up")
        _check_dev(orb_dn, torch.float64, (W, self.n_elec[1], 5, self.n_orb[1]), "orb_dn")
        la, sg = self._empty(W), self._empty(W)
        st = status if status is not None else torch.zeros(W, dtype=torch.int32, device=self.device)
        self.state_seq += 1
        self._chk(lib().mde_init(self._h, W, _ptr(orb_up), _ptr(orb_dn), _ptr(la), _ptr(sg),
                                 _ptr(st)), "init")
        return la, sg, st

    def refresh(self, status=None):
        W = self.W
        la, sg = self._empty(W), self._empty(W)
        st = status if status is not None else torch.zeros(W, dtype=torch.int32, device=self.device)
        self.state_seq += 1
        self._chk(lib().mde_refresh(self._h, _ptr(la), _ptr(sg), _ptr(st)), "refresh")
        return la, sg, st

    def spin_of(self, e: int) -> int:
        return 0 if e < self.n_elec[0] else 1

    def propose(self, e: int, new_orb: torch.Tensor, out=None):
        """Returns (ratio [W], grad [W,3], lap [W], status [W])."""
        W = self.W
        s = self.spin_of(e)
        _check_dev(new_orb, torch.float64, (W, 5, self.n_orb[s]), "new_orb")
        if out is None:
            out = (self._empty(W), self._empty((W, 3)), self._empty(W),
                   torch.zeros(W, dtype=torch.int32, device=self.device))
        r, g, l, st = out
        self.state_seq += 1
        self._chk(lib().mde_propose(self._h, e, _ptr(new_orb), _ptr(r), _ptr(g), _ptr(l), _ptr(st)),
                  "propose")
        return out

    def grad_lap(self, e: int, cur_orb: torch.Tensor, out=None):
        W = self.W
        s = self.spin_of(e)
        _check_dev(cur_orb, torch.float64, (W, 5, self.n_orb[s]), "cur_orb")
        if out is None:
            out = (self._empty((W, 3)), self._empty(W),
                   torch.zeros(W, dtype=torch.int32, device=self.device))
        g, l, st = out
        self.state_seq += 1
        self._chk(lib().mde_grad_lap(self._h, e, _ptr(cur_orb), _ptr(g), _ptr(l), _ptr(st)),
                  "grad_lap")
        return out

    def local_derivs(self, orb_up: torch.Tensor, orb_dn: torch.Tensor, out=None):
        """grad_i ln Psi [W, n_tot, 3] and lap_i Psi / Psi [W, n_tot] of every
        electron at the current positions; orb_* are every electron's blocks
        (as for init).  Returns (grad, lap, status)."""
        W = self.W
        _check_dev(orb_up, torch.float64, (W, self.n_elec[0], 5, self.n_orb[0]), "orb_up")
        _check_dev(orb_dn, torch.float64, (W, self.n_elec[1], 5, self.n_orb[1]), "orb_dn")
        nt = self.n_elec[0] + self.n_elec[1]
        if out is None:
            out = (self._empty((W, nt, 3)), self._empty((W, nt)),
                   torch.zeros(W, dtype=torch.int32, device=self.device))
        g, l, st = out
        self._chk(lib().mde_local_derivs(self._h, _ptr(orb_up), _ptr(orb_dn), _ptr(g), _ptr(l),
                                         _ptr(st)), "local_derivs")
        return out

    def vmc(self, n_steps: int, tau: float, normals: torch.Tensor, uniforms: torch.Tensor,
            pos: torch.Tensor, accepted: torch.Tensor, status=None):
        """n_steps Metropolis sweeps with drift on the device; pos [W, n_tot, 3]
        and accepted [W] (int32) are updated in place.  normals
        [n_steps, n_tot, W, 3] and uniforms [n_steps, n_tot, W] are the
        random inputs."""
        W, nt = self.W, self.n_elec[0] + self.n_elec[1]
        _check_dev(normals, torch.float64, (n_steps, nt, W, 3), "normals")
        _check_dev(uniforms, torch.float64, (n_steps, nt, W), "uniforms")
        _check_dev(pos, torch.float64, (W, nt, 3), "pos")
        _check_dev(accepted, torch.int32, (W,), "accepted")
        st = status if status is not None else torch.zeros(W, dtype=torch.int32, device=self.device)
        self.state_seq += 1
        self._chk(lib().mde_vmc(self._h, int(n_steps), float(tau), _ptr(normals), _ptr(uniforms),
                                _ptr(pos), _ptr(accepted), _ptr(st)), "vmc")
        return st

    def accept(self, e: int, mask: torch.Tensor):
        _check_dev(mask, torch.uint8, (self.W,), "accept mask")
        self.state_seq += 1
        self._chk(lib().mde_accept(self._h, e, _ptr(mask)), "accept")

    def export(self, what: str, spin: int = 0) -> torch.Tensor:
        W = self.W
        n, no = self.n_elec[spin], self.n_orb[spin]
        codes = {"inverse": (0, (W, n, n)), "table": (1, (W, n, no - n)),
                 "ratios": (2, (W, self._n_exc(spin))), "logdet": (3, (W,)), "N": (4, (W,))}
        code, shape = codes[what]
        out = self._empty(shape)
        self._chk(lib().mde_export(self._h, code, spin, _ptr(out)), "export")
        return out

    def _n_exc(self, spin):
        return self._nexc[spin]

    # -- adjoint ---------------------------------------------------------------------
    def eval_tables(self, T_up: torch.Tensor, T_dn: torch.Tensor, coef: torch.Tensor):
        W = self.W
        _check_dev(T_up, torch.float64, (W, self.n_elec[0], self.n_orb[0] - self.n_elec[0]), "T_up")
        _check_dev(T_dn, torch.float64, (W, self.n_elec[1], self.n_orb[1] - self.n_elec[1]), "T_dn")
        _check_dev(coef, torch.float64, (self.n_det,), "coef")
        la, sg = self._empty(W), self._empty(W)
        st = torch.zeros(W, dtype=torch.int32, device=self.device)
        self.state_seq += 1
        self._chk(lib().mde_eval_tables(self._h, W, _ptr(T_up), _ptr(T_dn), _ptr(coef), _ptr(la),
                                        _ptr(sg), _ptr(st)), "eval_tables")
        return la, sg, st

    def backward(self, go: torch.Tensor, want_coef=True, want_T=True, status=None):
        W = self.W
        _check_dev(go, torch.float64, (W,), "go")
        gc = self._empty(self.n_det) if want_coef else None
        gu = self._empty((W, self.n_elec[0], self.n_orb[0] - self.n_elec[0])) if want_T else None
        gd = self._empty((W, self.n_elec[1], self.n_orb[1] - self.n_elec[1])) if want_T else None
        self._chk(lib().mde_backward(self._h, _ptr(go), _ptr(gc), _ptr(gu), _ptr(gd), _ptr(status)),
                  "backward")
        return gc, gu, gd

    # -- tuning / graphs ------------------------------------------------------------
    def set_plan(self, spin: int, walker_tile: int = 0, item_exc: int = 0, threads: int = 0):
        self._chk(lib().mde_set_plan(self._h, spin, walker_tile, item_exc, threads), "set_plan")

    def get_plan(self, spin: int):
        a, b, c = C.c_int32(), C.c_int32(), C.c_int32()
        self._chk(lib().mde_get_plan(self._h, spin, C.byref(a), C.byref(b), C.byref(c)), "get_plan")
        return dict(walker_tile=a.value, item_exc=b.value, threads=c.value)

    def autotune(self, new_orb_up: torch.Tensor, new_orb_dn: torch.Tensor, cache_path=None):
        cp = cache_path.encode() if cache_path else None
        self._chk(lib().mde_autotune(self._h, _ptr(new_orb_up), _ptr(new_orb_dn), cp), "autotune")

    def profile_enable(self, max_launches: int, repeat: int = 1):
        self._chk(lib().mde_profile_enable(self._h, max_launches, repeat), "profile_enable")

    def profile_read(self):
        """(total ms, count) of the bracketed determinant-kernel launches."""
        t, n = C.c_double(), C.c_int32()
        self._chk(lib().mde_profile_read(self._h, C.byref(t), C.byref(n)), "profile_read")
        return t.value, n.value

    def profile_disable(self):
        self._chk(lib().mde_profile_disable(self._h), "profile_disable")

    @contextmanager
    def capture(self):
        """with ctx.capture() as cap: ...calls...;  cap.graph.launch()"""
        class _Cap:
            graph = None
        cap = _Cap()
        self._chk(lib().mde_capture_begin(self._h), "capture_begin")
        try:
            yield cap
        finally:
            h = C.c_void_p()
            self._chk(lib().mde_capture_end(self._h, C.byref(h)), "capture_end")
            cap.graph = Graph(h, self.stream)

    # -- synthetic orbitals -------------------------------------------------------------
    def sgauss_eval(self, spin: int, pos: torch.Tensor) -> torch.Tensor:
        _check_dev(pos, torch.float64, None, "pos")
        P = pos.numel() // 3
        out = self._empty(tuple(pos.shape[:-1]) + (5, self.n_orb[spin]))
        self._chk(lib().mde_sgauss_eval(self._h, spin, P, _ptr(pos), _ptr(out)), "sgauss_eval")
        return out

    # -- convenience -------------------------------------------------------------------
    def set_expansion(self, exc_up, exc_dn, coef, det_up, det_dn):
        """exc_*: objects with offsets/holes/particles arrays (CSR)."""
        self._nexc = (int(exc_up.offsets.shape[0] - 1), int(exc_dn.offsets.shape[0] - 1))
        self.set_excitations(0, exc_up.offsets, exc_up.holes, exc_up.particles)
        self.set_excitations(1, exc_dn.offsets, exc_dn.holes, exc_dn.particles)
        self.set_ci(coef, det_up, det_dn)


class Group:
    """Uneven batch: several contexts packed into one persistent launch.

    Pass contexts whose expansion is set but which are not bound yet, with
    their walker counts: the group gives them one common walker tile (the
    smallest of their defaults) and binds them.  Already-bound contexts must
    share a walker tile."""

    @staticmethod
    def prepare(ctxs: Sequence[Context], Ws: Sequence[int]):
        wt = min(min(c.get_plan(0)["walker_tile"], c.get_plan(1)["walker_tile"]) for c in ctxs)
        for c, W in zip(ctxs, Ws):
            for sp in (0, 1):
                c.set_plan(sp, walker_tile=wt)
            c.bind(W)
        return wt

    @staticmethod
    def by_tile(ctxs: Sequence[Context], Ws: Sequence[int]):
        """Unbound contexts split by their default walker tile (the smaller of
        their two spins'): one group, hence one launch, per tile size, so that
        instances with small tables keep wide tiles instead of all taking the
        narrowest.  Returns [(group, positions of its contexts in ctxs)]."""
        classes = {}
        for i, c in enumerate(ctxs):
            wt = min(c.get_plan(0)["walker_tile"], c.get_plan(1)["walker_tile"])
            classes.setdefault(wt, []).append(i)
        out = []
        for wt in sorted(classes, reverse=True):
            idx = classes[wt]
            out.append((Group([ctxs[i] for i in idx], [Ws[i] for i in idx]), idx))
        return out

    def __init__(self, ctxs: Sequence[Context], Ws: Optional[Sequence[int]] = None,
                 common_tile: bool = True):
        """Ws: bind the (unbound) contexts first, with one common walker tile
        (one launch for all) or, with common_tile=False, each with its own
        default tile (the library then runs one launch per tile class)."""
        if Ws is not None:
            if common_tile:
                Group.prepare(ctxs, Ws)
            else:
                for c, W in zip(ctxs, Ws):
                    c.bind(W)
        self.ctxs = list(ctxs)
        arr = (C.c_void_p * len(ctxs))(*[c._h.value for c in ctxs])
        self._arr = arr
        b = C.c_size_t()
        rc = lib().mde_group_workspace_bytes(arr, len(ctxs), C.byref(b))
        if rc:
            raise MdeError(rc, "group_workspace_bytes")
        dev = ctxs[0].device
        self.workspace = torch.empty(int(b.value) + 256, dtype=torch.uint8, device=dev)
        off = (-self.workspace.data_ptr()) % 256
        h = C.c_void_p()
        rc = lib().mde_group_create(arr, len(ctxs), self.workspace.data_ptr() + off, int(b.value),
                                    C.byref(h))
        if rc:
            raise MdeError(rc, "group_create")
        self._h = h
        self.stream = ctxs[0].stream

    def _chk(self, rc, what):
        if rc:
            msg = lib().mde_group_error_string(self._h)
            raise MdeError(rc, f"{what}: {msg.decode() if msg else ''}")

    def __del__(self):
        try:
            if getattr(self, "_h", None):
                lib().mde_group_destroy(self._h)
        except Exception:
            pass

    @staticmethod
    def _ptrs(ts):
        return (C.c_void_p * len(ts))(*[(t.data_ptr() if t is not None else None) for t in ts])

    def propose(self, es, new_orbs, outs):
        """outs: list of (ratio, grad, lap, status) per instance."""
        n = len(self.ctxs)
        e = np.ascontiguousarray(es, np.int32)
        self._keepalive = (self._ptrs(new_orbs), self._ptrs([o[0] for o in outs]),
                           self._ptrs([o[1] for o in outs]), self._ptrs([o[2] for o in outs]),
                           self._ptrs([o[3] for o in outs]), e)
        k = self._keepalive
        self._chk(lib().mde_group_propose(self._h, _np_ptr(e), k[0], k[1], k[2], k[3], k[4]),
                  "group_propose")

    def tune(self, es, new_orbs):
        """Autotune the members' launch plans on proposals of electrons es to
        new_orbs (the members' state is re-evaluated from their orbitals)."""
        e = np.ascontiguousarray(es, np.int32)
        arr = self._ptrs(new_orbs)
        self._chk(lib().mde_group_tune(self._h, _np_ptr(e), arr), "group_tune")
        for c in self.ctxs:
            c.state_seq += 1

    def accept(self, es, masks):
        e = np.ascontiguousarray(es, np.int32)
        arr = self._ptrs(masks)
        self._keep_acc = (arr, e)
        self._chk(lib().mde_group_accept(self._h, _np_ptr(e), arr), "group_accept")

    @contextmanager
    def capture(self):
        class _Cap:
            graph = None
        cap = _Cap()
        self._chk(lib().mde_group_capture_begin(self._h), "group_capture_begin")
        try:
            yield cap
        finally:
            h = C.c_void_p()
            self._chk(lib().mde_group_capture_end(self._h, C.byref(h)), "group_capture_end")
            cap.graph = Graph(h, self.stream)
