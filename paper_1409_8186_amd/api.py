"""Python binding of libmudiff (include/mudiff.h): argument marshalling only.

PyTorch supplies the device memory (tensors) and the stream (the current
torch stream); every computation runs in the HIP kernels behind the C ABI.

Vectors are flat complex128 tensors packed [B][R][N_b] (instance, right-hand
side, unknown), unknowns of an instance ordered disk by disk with modes
m = -N_p..N_p.  ``Problem.split`` / ``Problem.pack`` convert to and from a list
of [R, N_b] tensors.
"""
from __future__ import annotations

import ctypes
from typing import Sequence

import numpy as np
import torch

from . import _lib as L


def _p(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _host(a, dtype):
    return np.ascontiguousarray(np.asarray(a, dtype=dtype))


class Problem:
    """B independent disk clusters sharing one set of device tables.

    ``instances``: sequence of (centers [M,2], radii [M], n_modes [M], k).
    ``circulant``: also build the circulant-embedded form of the well-separated
    blocks (MUDIFF_TABLES_CIRCULANT), used by multi-right-hand-side applies.
    """

    def __init__(self, instances: Sequence, device: str = "cuda", circulant: bool = False):
        self.lib = L.load()
        if not torch.cuda.is_available():
            raise RuntimeError("libmudiff needs a HIP device")
        self.device = torch.device(device)
        cs, rs, ns, ks, offs = [], [], [], [], [0]
        for (c, r, n, k) in instances:
            c = _host(c, np.float64).reshape(-1, 2)
            cs.append(c)
            rs.append(_host(r, np.float64).reshape(-1))
            ns.append(_host(n, np.int32).reshape(-1))
            ks.append(float(k))
            offs.append(offs[-1] + c.shape[0])
        self.B = len(ks)
        self.centers = np.ascontiguousarray(np.concatenate(cs))
        self.radii = np.ascontiguousarray(np.concatenate(rs))
        self.n_modes = np.ascontiguousarray(np.concatenate(ns))
        self.k = _host(ks, np.float64)
        self.disk_off = _host(offs, np.int64)
        self.flags = L.TABLES_CIRCULANT if circulant else 0
        ws = self.lib.mudiff_tables_workspace_size(self.B, self.disk_off.ctypes.data,
                                                   self.n_modes.ctypes.data, self.flags)
        if ws == 0:
            raise L.MudiffError(1, "invalid sizes (disk_off / n_modes)")
        self.ws = torch.empty(int(ws), dtype=torch.uint8, device=self.device)
        assert self.ws.data_ptr() % 256 == 0
        h = ctypes.c_void_p()
        L.check(self.lib.mudiff_tables(self.B, self.disk_off.ctypes.data, self.centers.ctypes.data,
                                       self.radii.ctypes.data, self.n_modes.ctypes.data,
                                       self.k.ctypes.data, _p(self.ws), int(ws), self.flags,
                                       _stream(), ctypes.byref(h)))
        self.h = h
        n = np.zeros(self.B, np.int64)
        L.check(self.lib.mudiff_sizes(h, n.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))))
        self.n_tot = n
        self.N_all = int(n.sum())
        self._mv_ws = {}

    @classmethod
    def from_cluster(cls, cl, device="cuda", circulant=False):
        return cls([(cl.centers, cl.radii, cl.n_modes, cl.k)], device, circulant)

    @classmethod
    def from_clusters(cls, cls_list, device="cuda", circulant=False):
        return cls([(c.centers, c.radii, c.n_modes, c.k) for c in cls_list], device, circulant)

    def close(self):
        if getattr(self, "h", None):
            self.lib.mudiff_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ----------------------------------------------------------- layout helpers
    def empty(self, R: int = 1) -> torch.Tensor:
        return torch.empty(R * self.N_all, dtype=torch.complex128, device=self.device)

    def split(self, v: torch.Tensor, R: int = 1) -> list:
        out, o = [], 0
        for b in range(self.B):
            n = int(self.n_tot[b])
            out.append(v[o:o + R * n].view(R, n))
            o += R * n
        return out

    def pack(self, parts) -> torch.Tensor:
        return torch.cat([torch.as_tensor(p).reshape(-1) for p in parts]).to(
            self.device, torch.complex128).contiguous()

    def _f64(self, a) -> torch.Tensor:
        if isinstance(a, torch.Tensor):
            return a.to(self.device, torch.float64).contiguous()
        return torch.as_tensor(np.asarray(a, dtype=np.float64)).to(self.device).contiguous()

    # ----------------------------------------------------------- tables
    def disk_tables(self):
        D = int(np.sum(self.n_modes + 2))
        J = torch.empty(D, dtype=torch.float64, device=self.device)
        H = torch.empty(D, dtype=torch.complex128, device=self.device)
        L.check(self.lib.mudiff_disk_tables(self.h, _p(J), _p(H), _stream()))
        return J, H

    def pair_tables(self):
        cnt = ctypes.c_int64()
        L.check(self.lib.mudiff_pair_tables(self.h, None, ctypes.byref(cnt), _stream()))
        t = torch.empty(max(cnt.value, 1), dtype=torch.complex128, device=self.device)
        L.check(self.lib.mudiff_pair_tables(self.h, _p(t), ctypes.byref(cnt), _stream()))
        return t[:cnt.value]

    # ----------------------------------------------------------- operator
    def matvec_workspace(self, R: int) -> torch.Tensor:
        if R not in self._mv_ws:
            n = self.lib.mudiff_matvec_workspace_size(self.h, R)
            # zero once: the library leaves its counters at zero after every call
            self._mv_ws[R] = torch.zeros(int(n), dtype=torch.uint8, device=self.device)
        return self._mv_ws[R]

    def matvec(self, x: torch.Tensor, R: int = 1, op: int = L.OP_A, out=None) -> torch.Tensor:
        x = x.contiguous()
        assert x.dtype == torch.complex128 and x.numel() == R * self.N_all
        y = self.empty(R) if out is None else out
        ws = self.matvec_workspace(R)
        L.check(self.lib.mudiff_matvec(self.h, R, _p(x), _p(y), op, _p(ws), ws.numel(), _stream()))
        return y

    def apply_config(self, R: int = 1) -> dict:
        """Kernel configuration of the R-column apply on this handle
        (kind: lane / mfma / generic; MFMA tile and autotuned time)."""
        vals = [ctypes.c_int(0) for _ in range(5)]
        ms = ctypes.c_float(0.0)
        L.check(self.lib.mudiff_apply_config(self.h, R, *[ctypes.byref(v) for v in vals],
                                              ctypes.byref(ms)))
        kind, ct, rp, qs, th = (v.value for v in vals)
        return {"kind": ["lane", "mfma", "generic", "circulant"][kind], "ct": ct, "rp": rp,
                "qs": qs, "threads": th, "tuned_ms": ms.value}

    def set_apply_config(self, R: int, ct: int, rp: int, qs: int, threads: int) -> None:
        """Fix the MFMA tile of the R-column apply (no autotuning for this R)."""
        L.check(self.lib.mudiff_set_apply_config(self.h, R, ct, rp, qs, threads))

    def circulant_info(self) -> dict:
        """Ordered pairs in the circulant (well-separated) and direct (close)
        forms, and the largest embedding length."""
        far, near, lm = ctypes.c_int64(0), ctypes.c_int64(0), ctypes.c_int(0)
        L.check(self.lib.mudiff_circulant_info(self.h, ctypes.byref(far), ctypes.byref(near),
                                               ctypes.byref(lm)))
        return {"far_pairs": far.value, "near_pairs": near.value, "L_max": lm.value}

    def set_circulant(self, R: int, mode: int) -> None:
        """Form of the R-column apply: -1 timed, 0 direct only, 1 circulant."""
        L.check(self.lib.mudiff_set_circulant(self.h, R, mode))

    # per-frequency product tiles (rows, cols, kstep, stages, threads, real products per
    # complex product) timed for R
    CIRCULANT_TILES = {48: [(64, 32, 16, 2, 256, 4), (64, 32, 16, 3, 256, 4), (128, 32, 16, 2, 512, 4),
                            (128, 32, 16, 3, 512, 4), (128, 32, 8, 3, 512, 4), (128, 32, 8, 2, 512, 4),
                            (64, 32, 8, 3, 256, 4), (128, 64, 8, 3, 512, 4), (128, 64, 16, 3, 512, 4),
                            (128, 32, 4, 2, 512, 4), (128, 32, 8, 2, 1024, 4), (64, 32, 8, 2, 256, 4),
                            (256, 32, 8, 2, 512, 4), (128, 32, 8, 2, 512, 3), (128, 32, 16, 2, 512, 3),
                            (128, 32, 8, 3, 512, 3), (128, 64, 8, 2, 512, 3), (256, 32, 8, 2, 512, 3),
                            (64, 32, 8, 2, 256, 3)],
                       24: [(64, 32, 16, 2, 256, 4), (64, 32, 32, 2, 256, 4), (128, 32, 16, 2, 256, 4),
                            (64, 32, 16, 3, 256, 4), (128, 32, 16, 2, 512, 4), (128, 32, 16, 3, 512, 4),
                            (128, 32, 8, 3, 512, 4), (128, 32, 8, 2, 512, 4), (64, 32, 8, 3, 256, 4),
                            (64, 32, 8, 2, 256, 4), (128, 32, 8, 2, 512, 3), (128, 32, 16, 2, 512, 3),
                            (64, 32, 8, 2, 256, 3)],
                       12: [(128, 16, 16, 2, 256, 4), (128, 8, 16, 2, 256, 4), (128, 16, 16, 3, 256, 4),
                            (128, 16, 8, 2, 256, 4), (128, 16, 8, 2, 256, 3), (128, 16, 16, 2, 256, 3)],
                       1: [(128, 8, 16, 2, 256, 4), (64, 8, 16, 2, 256, 4), (128, 8, 8, 2, 256, 4)]}

    @classmethod
    def circulant_tiles(cls, R: int) -> list:
        """Per-frequency product tiles (rows, cols, kstep, stages, threads) timed for R."""
        for lo in (48, 24, 12, 1):
            if R >= lo:
                return cls.CIRCULANT_TILES[lo]

    def profile_begin(self, max_applies: int) -> None:
        """Record HIP events between the phases of the next max_applies applies."""
        L.check(self.lib.mudiff_profile_begin(self.h, max_applies))

    def profile_end(self) -> dict:
        """{"applies": n, phase: summed ms} of the applies profiled since profile_begin."""
        n = ctypes.c_int(0)
        ms = (ctypes.c_double * L.N_PHASES)()
        L.check(self.lib.mudiff_profile_end(self.h, ctypes.byref(n), ms))
        out = {"applies": n.value}
        out.update({name: ms[k] for k, name in enumerate(L.PHASES)})
        return out

    def circulant_tile(self, R: int) -> tuple:
        v = [ctypes.c_int(0) for _ in range(6)]
        L.check(self.lib.mudiff_circulant_tile(self.h, R, *[ctypes.byref(x) for x in v]))
        return tuple(x.value for x in v)

    def set_circulant_tile(self, R: int, rows: int, cols: int, kstep: int, stages: int,
                           threads: int, mults: int = 4) -> None:
        L.check(self.lib.mudiff_set_circulant_tile(self.h, R, rows, cols, kstep, stages, threads,
                                                   mults))

    def rhs(self, betas=None, precond: bool = False, sources=None) -> torch.Tensor:
        """betas: [B, R] incidence angles, or sources: [B, R, 2] point-source
        positions (Prop. 5)."""
        if sources is not None:
            src = self._sources(sources)
            R = src.shape[1]
            out = self.empty(R)
            L.check(self.lib.mudiff_rhs_point(self.h, R, _p(src), _p(out), int(precond), _stream()))
            return out
        b = self._f64(betas).reshape(self.B, -1)
        R = b.shape[1]
        out = self.empty(R)
        L.check(self.lib.mudiff_rhs(self.h, R, _p(b), _p(out), int(precond), _stream()))
        return out

    def _sources(self, sources) -> torch.Tensor:
        return self._f64(sources).reshape(self.B, -1, 2).contiguous()

    # ----------------------------------------------------------- solver
    def gmres_workspace(self, R: int, restart: int, flags: int = 0) -> torch.Tensor:
        n = self.lib.mudiff_gmres_workspace_size(self.h, R, restart, flags)
        if n == 0:
            raise L.MudiffError(1, "invalid gmres sizes")
        return torch.empty(int(n), dtype=torch.uint8, device=self.device)

    def gmres(self, betas=None, rhs=None, R: int | None = None, restart: int = 50,
              tol: float = 1e-8, maxit: int = 20000, x0=None, graph: bool = False,
              want_resvec: bool = False, workspace=None, sources=None, precond: bool = True,
              block: int = 0, sstep: int = 0):
        """Solves L rho = -U for plane waves (betas [B, R]), point sources
        (sources [B, R, 2]) or a given U (rhs), with the single-scattering
        preconditioner unless precond=False; block > 0 runs block GMRES with
        blocks of that many consecutive columns, sstep > 0 s-step GMRES with
        that many Newton vectors per block.  Returns (rho, flag, relres,
        iters, resvec)."""
        flags = 0 if precond else L.NO_PRECOND
        if block:
            flags |= L.BLOCK | L.block_size(block)
        if sstep:
            flags |= L.SSTEP | L.sstep_size(sstep)
        bt = None
        if sources is not None:
            bt = self._sources(sources)
            R = bt.shape[1]
            flags |= L.POINT_SOURCE
        elif betas is not None:
            bt = self._f64(betas).reshape(self.B, -1)
            R = bt.shape[1]
        else:
            assert rhs is not None and R is not None
            rhs = rhs.contiguous()
        rho = self.empty(R)
        if x0 is not None:
            rho.copy_(x0)
            flags |= L.X0
        if graph:
            flags |= L.GRAPH
        ws = workspace if workspace is not None else self.gmres_workspace(R, restart, flags)
        C = self.B * R
        flag = torch.empty(C, dtype=torch.int32, device=self.device)
        relres = torch.empty(C, dtype=torch.float64, device=self.device)
        iters = torch.empty(C, dtype=torch.int32, device=self.device)
        resvec = (torch.empty(C * (maxit + 1), dtype=torch.float64, device=self.device)
                  if want_resvec else None)
        L.check(self.lib.mudiff_gmres(self.h, R, _p(bt), _p(rhs), _p(rho), restart, tol, maxit,
                                      flags, _p(ws), ws.numel(), _p(flag), _p(relres), _p(iters),
                                      _p(resvec), _stream()))
        if resvec is not None:
            resvec = resvec.view(C, maxit + 1)
        return rho, flag, relres, iters, resvec

    # ----------------------------------------------------------- far field
    def farfield(self, rho: torch.Tensor, thetas, R: int = 1) -> torch.Tensor:
        th = self._f64(thetas).reshape(-1)
        out = torch.empty(self.B * R * th.numel(), dtype=torch.complex128, device=self.device)
        L.check(self.lib.mudiff_farfield(self.h, R, _p(rho.contiguous()), th.numel(), _p(th),
                                         _p(out), _stream()))
        return out.view(self.B * R, th.numel())

    # ----------------------------------------------------------- near field
    def nearfield(self, rho: torch.Tensor, points, R: int = 1, betas=None, sources=None) -> torch.Tensor:
        """Scattered field (or, with betas [B, R] or point sources [B, R, 2], the
        total field) at points [P, 2]; 0 inside disks.  Returns [B*R, P]."""
        pts = self._f64(points).reshape(-1, 2).contiguous()
        flags = 0
        if sources is not None:
            bt = self._f64(sources).reshape(self.B, R, 2).contiguous()
            flags = L.POINT_SOURCE
        else:
            bt = None if betas is None else self._f64(betas).reshape(self.B, R).contiguous()
        out = torch.empty(self.B * R * pts.shape[0], dtype=torch.complex128, device=self.device)
        L.check(self.lib.mudiff_nearfield(self.h, R, _p(rho.contiguous()), pts.shape[0], _p(pts),
                                          _p(bt), flags, _p(out), _stream()))
        return out.view(self.B * R, pts.shape[0])

    # ----------------------------------------------------------- operators
    FORMULATIONS = ("efie", "mfie", "cfie", "bwie", "neumann_sl", "neumann_dl")

    def set_operator(self, name: str | None = None, ops=None, rhs=None, far=None,
                     alpha: float = 0.5, eta: complex | None = None) -> None:
        """Solve, apply and evaluate far fields with another formulation: a name
        of FORMULATIONS (mudiff_set_formulation; eta defaults to i k of the first
        instance), or explicit weight dicts over I, L, M, N, D / U, dU / L, M
        (mudiff_set_operator); None returns to the built-in single layer."""
        n = self.lib.mudiff_operator_workspace_size(self.h)
        if name is None and ops is None:
            L.check(self.lib.mudiff_set_operator(self.h, None, None, None, None, 0, _stream()))
            self._op_ws = None
            return
        ws = torch.empty(int(n), dtype=torch.uint8, device=self.device)
        if name is not None:
            if eta is None:
                eta = 1j * float(self.k[0])
            eta = complex(eta)
            kind = self.FORMULATIONS.index(name)
            L.check(self.lib.mudiff_set_formulation(self.h, kind, float(alpha), eta.real, eta.imag,
                                                    _p(ws), ws.numel(), _stream()))
            self._op_ws = ws if name != "efie" else None
            return

        def cvec(d, keys):
            out = np.zeros(2 * len(keys), dtype=np.float64)
            for i, key in enumerate(keys):
                v = complex(d.get(key, 0.0))
                out[2 * i], out[2 * i + 1] = v.real, v.imag
            return out
        w = cvec(ops, "ILMND")
        rw = cvec(rhs or {}, ("U", "dU"))
        fw = cvec(far or {"L": 1.0}, ("L", "M"))
        L.check(self.lib.mudiff_set_operator(self.h, w.ctypes.data, rw.ctypes.data, fw.ctypes.data,
                                             _p(ws), ws.numel(), _stream()))
        self._op_ws = ws  # the handle points into it

    def set_penetrable(self, k_int, mu=None) -> None:
        """Penetrable disks (sec. 7, Example II): interior wavenumber k_int and
        contrast mu (scalars or one per disk over all instances).  gmres then
        returns the exterior density rho+, farfield/nearfield the scattered field;
        set_operator(None) returns to sound-soft disks."""
        ki = np.broadcast_to(np.asarray(k_int, dtype=np.float64), (len(self.radii),)).copy()
        mu_a = None if mu is None else np.broadcast_to(np.asarray(mu, dtype=np.float64), (len(self.radii),)).copy()
        n = self.lib.mudiff_operator_workspace_size(self.h)
        ws = torch.empty(int(n), dtype=torch.uint8, device=self.device)
        L.check(self.lib.mudiff_set_penetrable(self.h, ki.ctypes.data,
                                               None if mu_a is None else mu_a.ctypes.data,
                                               _p(ws), ws.numel(), _stream()))
        self._op_ws = ws

    def interior_field(self, rho: torch.Tensor, points, R: int = 1, betas=None, sources=None,
                       out=None) -> torch.Tensor:
        """Field inside penetrable disks (after set_penetrable and a solve for
        rho+ with these betas [B, R] or sources [B, R, 2]) at points [P, 2],
        written into out [B*R, P] (a fresh zero tensor if None) at the points
        inside a disk; other points keep their values."""
        pts = self._f64(points).reshape(-1, 2).contiguous()
        if sources is not None:
            inc, flags = self._f64(sources).reshape(self.B, R, 2).contiguous(), L.POINT_SOURCE
        else:
            inc, flags = self._f64(betas).reshape(self.B, R).contiguous(), 0
        if out is None:
            out = torch.zeros(self.B * R, pts.shape[0], dtype=torch.complex128, device=self.device)
        assert out.is_contiguous() and out.numel() == self.B * R * pts.shape[0]
        n = self.lib.mudiff_interior_workspace_size(self.h, R)
        ws = torch.empty(int(n), dtype=torch.uint8, device=self.device)
        L.check(self.lib.mudiff_interior_field(self.h, R, _p(rho.contiguous()), _p(inc), flags,
                                               pts.shape[0], _p(pts), _p(out), _p(ws), ws.numel(),
                                               _stream()))
        return out

    # ----------------------------------------------------------- time reversal
    def mirror_farfield(self, n_alpha: int, restart: int = 50, tol: float = 1e-12,
                        maxit: int = 20000, graph: bool = False):
        """Far-field matrix of a mirror with n_alpha cells (sec. 7, Example III):
        incidences alpha_j = 2 pi j / n_alpha, receivers at alpha_i + pi.  One
        instance only.  Returns (X, flag, relres, iters) with X[j, i] = F[i, j] =
        a(alpha_i + pi; alpha_j), shape [n_alpha, n_alpha]."""
        if self.B != 1:
            raise ValueError("mirror_farfield takes a handle with one instance")
        al = 2.0 * np.pi * np.arange(n_alpha) / n_alpha
        rho, flag, relres, iters, _ = self.gmres(betas=al[None, :], restart=restart, tol=tol,
                                                 maxit=maxit, graph=graph)
        X = self.farfield(rho, al + np.pi, R=n_alpha)
        return X, flag, relres, iters

    # ----------------------------------------------------------- gradient
    def grad_workspace(self, R: int, n_rec: int, restart: int, flags: int = 0) -> torch.Tensor:
        n = self.lib.mudiff_grad_workspace_size(self.h, R, n_rec, restart, flags)
        if n == 0:
            raise L.MudiffError(1, "invalid grad sizes")
        return torch.empty(int(n), dtype=torch.uint8, device=self.device)

    def grad(self, betas, thetas, target, restart: int = 50, tol: float = 1e-12,
             maxit: int = 20000, flags: int = 0, workspace=None):
        """Far-field misfit per instance and its gradient w.r.t. centers, radii, k.
        target: [B*R, n_rec] complex.  Returns (loss[B], d_centers[M,2], d_radii[M], d_k[B])."""
        bt = self._f64(betas).reshape(self.B, -1)
        R = bt.shape[1]
        th = self._f64(thetas).reshape(-1)
        tg = torch.as_tensor(target).to(self.device, torch.complex128).contiguous()
        assert tg.numel() == self.B * R * th.numel()
        ws = workspace if workspace is not None else self.grad_workspace(R, th.numel(), restart, flags)
        M = self.radii.shape[0]
        loss = torch.empty(self.B, dtype=torch.float64, device=self.device)
        dc = torch.empty(M * 2, dtype=torch.float64, device=self.device)
        da = torch.empty(M, dtype=torch.float64, device=self.device)
        dk = torch.empty(self.B, dtype=torch.float64, device=self.device)
        L.check(self.lib.mudiff_grad(self.h, R, _p(bt), th.numel(), _p(th), _p(tg), restart, tol,
                                     maxit, flags, _p(ws), ws.numel(), _p(loss), _p(dc), _p(da),
                                     _p(dk), _stream()))
        return loss, dc.view(M, 2), da, dk


def probe(kind: str, nbytes: int = 1 << 30, device: str = "cuda") -> float:
    """Achievable device throughput: kind "fp64_fma" or "fp64_mfma" (TFLOP/s),
    or "copy" (GB/s of read + write over an nbytes copy).  Synchronises."""
    k = {"fp64_fma": L.PROBE_FP64_FMA, "fp64_mfma": L.PROBE_FP64_MFMA, "copy": L.PROBE_COPY}[kind]
    lib = L.load()
    n = lib.mudiff_probe_workspace_size(k, nbytes)
    if n == 0:
        raise L.MudiffError(1, "probe: no device or bad kind")
    ws = torch.empty(int(n), dtype=torch.uint8, device=device)
    rate = ctypes.c_double(0.0)
    L.check(lib.mudiff_probe(k, nbytes, _p(ws), ws.numel(), ctypes.byref(rate), _stream()))
    return rate.value


def tro(X: torch.Tensor) -> torch.Tensor:
    """T = conj(F)^T F for X = F^T ([n, m] complex128 on the device): T[a, b] =
    sum_i conj(X[a, i]) X[b, i]."""
    X = X.contiguous()
    n, m = X.shape
    lib = L.load()
    T = torch.empty(n, n, dtype=torch.complex128, device=X.device)
    L.check(lib.mudiff_tro(n, m, _p(X), _p(T), _stream()))
    return T


def tro_eigh(X: torch.Tensor, tol: float = 1e-13, max_sweeps: int = 60):
    """Eigenvalues (decreasing) and unit eigenvectors (rows) of T = conj(F)^T F
    from X = F^T by one-sided Jacobi; X is not modified.  Returns (w, evec, sweeps)."""
    Xw = X.contiguous().clone()
    n, m = Xw.shape
    lib = L.load()
    w = torch.empty(n, dtype=torch.float64, device=Xw.device)
    ev = torch.empty(n, n, dtype=torch.complex128, device=Xw.device)
    ws = torch.empty(int(lib.mudiff_tro_eigh_workspace_size(n, m)), dtype=torch.uint8,
                     device=Xw.device)
    sweeps = ctypes.c_int32(0)
    L.check(lib.mudiff_tro_eigh(n, m, _p(Xw), _p(w), _p(ev), max_sweeps, tol, _p(ws), ws.numel(),
                                ctypes.byref(sweeps), _stream()))
    return w, ev, sweeps.value


def herglotz(alpha, f: torch.Tensor, k: float, points, h: float | None = None) -> torch.Tensor:
    """u_t(x) = sum_j h f[t, j] exp(i k (x_1 cos alpha_j + x_2 sin alpha_j)) at
    points [P, 2]; f [n_f, n_alpha] (or [n_alpha]); h defaults to 2 pi / n_alpha."""
    dev = f.device
    al = torch.as_tensor(alpha, dtype=torch.float64).to(dev).contiguous()
    F = f.reshape(-1, al.numel()).to(torch.complex128).contiguous()
    pts = torch.as_tensor(points, dtype=torch.float64).to(dev).reshape(-1, 2).contiguous()
    h = 2.0 * np.pi / al.numel() if h is None else h
    u = torch.empty(F.shape[0], pts.shape[0], dtype=torch.complex128, device=dev)
    lib = L.load()
    L.check(lib.mudiff_herglotz(al.numel(), _p(al), F.shape[0], _p(F), float(k), float(h),
                                pts.shape[0], _p(pts), _p(u), _stream()))
    return u
