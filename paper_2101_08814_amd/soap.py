"""Python binding of the C ABI: argument marshalling only.

Every numerical step runs in the HIP kernels of libsoap_mi355x.so; torch
supplies device memory and the current stream.  Names follow the C entry
points (soap_compute_neighbors -> Calculator.compute_neighbors, ...).
"""
from __future__ import annotations

import ctypes
import os
import dataclasses
from typing import Optional

import numpy as np
import torch

from . import _lib
from ._lib import SOAP_BF16_F32ACC, SOAP_F32, SOAP_F64, check, soap_exec, soap_hypers, soap_table_info


def _ptr(t: Optional[torch.Tensor]):
    if t is None:
        return None
    return ctypes.c_void_p(t.data_ptr())


def _np_ptr(a: Optional[np.ndarray]):
    if a is None:
        return None
    return ctypes.c_void_p(a.ctypes.data)


def _precision(dtype) -> int:
    if dtype in (torch.float64, "f64", SOAP_F64):
        return SOAP_F64
    if dtype in (torch.float32, "f32", SOAP_F32):
        return SOAP_F32
    if dtype in ("bf16", SOAP_BF16_F32ACC):
        return SOAP_BF16_F32ACC
    raise ValueError(f"unsupported precision {dtype!r}")


def _torch_dtype(prec: int):
    return torch.float64 if prec == SOAP_F64 else torch.float32


@dataclasses.dataclass
class Neighbors:
    """Device neighbour list (CSR over centres)."""
    pair_offsets: torch.Tensor   # int64 [N+1]
    pair_j: torch.Tensor         # int32 [P]
    pair_shift: torch.Tensor     # int32 [P, 3]
    pair_vec: torch.Tensor       # float [P, 3]
    pair_transpose: Optional[torch.Tensor]  # int32 [P]
    n_pairs: int

    @property
    def capacity(self) -> int:
        return int(self.pair_j.shape[0])

    def count(self) -> int:
        """Number of pairs (reads pair_offsets[N] from the device)."""
        if self.n_pairs < 0:
            self.n_pairs = int(self.pair_offsets[-1].item())
        return self.n_pairs


class Calculator:
    """Owns a soap_calculator (hyper-parameters + spline tables)."""

    def __init__(self, n_species: int, nmax: int, lmax: int, rcut: float, sigma: float,
                 cutoff_width: float = 0.5, include_center: int = 1, spline_accuracy: float = 1e-8,
                 radial_basis=0):
        """radial_basis: 0 or "gto" (orthogonalised GTOs), 1 or "dvr"."""
        self._L = _lib.lib()
        basis = {"gto": _lib.SOAP_RADIAL_GTO, "dvr": _lib.SOAP_RADIAL_DVR}.get(radial_basis, radial_basis)
        h = soap_hypers(int(n_species), int(nmax), int(lmax), int(include_center), float(rcut),
                        float(cutoff_width), float(sigma), float(spline_accuracy), int(basis), 0)
        handle = ctypes.c_void_p()
        check(self._L.soap_calculator_create(ctypes.byref(h), ctypes.byref(handle)))
        self.handle = handle
        self.hypers = dict(n_species=int(n_species), nmax=int(nmax), lmax=int(lmax), rcut=float(rcut),
                           sigma=float(sigma), cutoff_width=float(cutoff_width),
                           include_center=int(include_center), spline_accuracy=float(spline_accuracy),
                           radial_basis=int(basis))
        self.S, self.nmax, self.lmax = int(n_species), int(nmax), int(lmax)
        self.L2 = (self.lmax + 1) ** 2
        self.K = self.S * self.nmax
        self.KK = self.K * (self.K + 1) // 2
        self._status = None
        self._ws = None

    @classmethod
    def from_hypers(cls, h: dict) -> "Calculator":
        return cls(h["n_species"], h["nmax"], h["lmax"], h["rcut"], h["sigma"], h.get("cutoff_width", 0.5),
                   h.get("include_center", 1), h.get("spline_accuracy", 1e-8), h.get("radial_basis", 0))

    def __del__(self):
        try:
            if getattr(self, "handle", None) is not None and self.handle.value:
                self._L.soap_calculator_destroy(self.handle)
                self.handle = None
        except Exception:
            pass

    # ------------------------------------------------------------ host info
    def info(self) -> dict:
        inf = soap_table_info()
        check(self._L.soap_calculator_info(self.handle, ctypes.byref(inf)))
        return {k: getattr(inf, k) for k, _ in soap_table_info._fields_}

    def radial_integral_host(self, r, exact: bool = False):
        r = np.ascontiguousarray(np.atleast_1d(r), dtype=np.float64)
        I = np.zeros((r.shape[0], self.nmax, self.lmax + 1))
        dI = np.zeros_like(I)
        check(self._L.soap_radial_integral_host(self.handle, int(exact), r.shape[0], _np_ptr(r), _np_ptr(I),
                                                _np_ptr(dI)))
        return I, dI

    def radial_integral(self, r: torch.Tensor, exact: bool = False, dtype=torch.float64, deriv: bool = True):
        """soap_radial_integral on the device: I~_nl(r_k) (and d/dr) as
        [nmax, lmax+1, n_r] tensors, from the spline (exact=False) or
        evaluated directly (exact=True, FP64)."""
        assert r.dtype == torch.float64 and r.is_cuda
        r = r.contiguous()
        prec = _precision(dtype)
        td = _torch_dtype(prec)
        n = int(r.shape[0])
        I = torch.empty((self.nmax, self.lmax + 1, max(n, 1)), dtype=td, device=r.device)
        dI = torch.empty_like(I) if deriv else None
        e = self._exec()
        check(self._L.soap_radial_integral(self.handle, ctypes.byref(e), prec, int(bool(exact)), n, _ptr(r), _ptr(I),
                                           _ptr(dI)))
        return (I[..., :n], dI[..., :n]) if deriv else I[..., :n]

    # ------------------------------------------------------------ execution
    def _exec(self, status: Optional[torch.Tensor] = None, device=None) -> soap_exec:
        stream = torch.cuda.current_stream(device).cuda_stream
        if status is None:
            if self._status is None or self._status.device != torch.device("cuda", torch.cuda.current_device()):
                self._status = torch.zeros(1, dtype=torch.int32, device="cuda")
            status = self._status
        return soap_exec(ctypes.c_void_p(stream), ctypes.c_void_p(status.data_ptr()))

    def reset_status(self):
        if self._status is not None:
            self._status.zero_()

    def device_status(self) -> int:
        """Synchronises the current stream and returns the device status word."""
        e = self._exec()
        return int(self._L.soap_read_device_status(ctypes.byref(e)))

    def check_device(self):
        """Raises SoapError if a kernel stored an error in the status word."""
        st = self.device_status()
        if st != 0:
            raise _lib.SoapError(st, "reported by a kernel in the device status word")

    def neighbors_workspace_size(self, n_structures: int, n_atoms: int) -> int:
        n = ctypes.c_size_t()
        check(self._L.soap_neighbors_workspace_size(self.handle, int(n_structures), int(n_atoms), ctypes.byref(n)))
        return int(n.value)

    def compute_neighbors(self, positions: torch.Tensor, species: torch.Tensor, atom_offsets, cells, pbc,
                          vec_dtype=torch.float32, capacity: Optional[int] = None, transpose: bool = True,
                          out: Optional[Neighbors] = None) -> Neighbors:
        """soap_compute_neighbors.  atom_offsets, cells and pbc may be host
        arrays (copied to the device here) or device tensors (used as they
        are; then the call copies nothing and can be graph-captured).  With
        capacity None the list is sized exactly: a counting call, one 8-byte
        read of the total, a filling call.  With out given, its buffers are
        refilled in place."""
        dev = positions.device
        ao, ce, pb = structures_to_device(atom_offsets, cells, pbc, dev)
        N = int(positions.shape[0])
        n_struct = int(ao.shape[0] - 1)
        assert positions.dtype == torch.float64 and positions.is_cuda and positions.shape == (N, 3)
        assert species.dtype == torch.int32 and species.is_cuda and species.shape == (N,)
        positions = positions.contiguous()
        species = species.contiguous()
        ws_bytes = self.neighbors_workspace_size(n_struct, N)
        if self._ws is None or self._ws.numel() < ws_bytes or self._ws.device != dev:
            self._ws = torch.empty(max(ws_bytes, 256), dtype=torch.uint8, device=dev)
        prec = _precision(vec_dtype)
        args = (n_struct, N, ao, ce, pb, positions, species)
        if out is not None:
            self._call_neighbors(*args, out.capacity, prec, out.pair_offsets, out.pair_j, out.pair_shift,
                                 out.pair_vec, out.pair_transpose)
            return out
        offsets = torch.empty(N + 1, dtype=torch.int64, device=dev)
        exact = capacity is None
        if exact:
            self._call_neighbors(*args, 0, prec, offsets, None, None, None, None)
            capacity = int(offsets[-1].item())
            self.reset_status()
        cap = max(int(capacity), 1)
        pj = torch.empty(cap, dtype=torch.int32, device=dev)
        ps = torch.empty((cap, 3), dtype=torch.int32, device=dev)
        pv = torch.empty((cap, 3), dtype=_torch_dtype(prec), device=dev)
        pt = torch.empty(cap, dtype=torch.int32, device=dev) if transpose else None
        self._call_neighbors(*args, cap, prec, offsets, pj, ps, pv, pt)
        return Neighbors(offsets, pj, ps, pv, pt, int(capacity) if exact else -1)

    def _call_neighbors(self, n_struct, N, ao, ce, pb, positions, species, capacity, prec, offsets, pj, ps, pv, pt):
        e = self._exec()
        check(self._L.soap_compute_neighbors(self.handle, ctypes.byref(e), n_struct, N, _ptr(ao), _ptr(ce), _ptr(pb),
                                             _ptr(positions), _ptr(species), _ptr(self._ws), self._ws.numel(),
                                             int(capacity), prec, _ptr(offsets), _ptr(pj), _ptr(ps), _ptr(pv),
                                             _ptr(pt)))

    def spherical_expansion(self, nl: Neighbors, species: torch.Tensor, dtype=torch.float32, gradients=False):
        prec = _precision(dtype)
        N = nl.pair_offsets.shape[0] - 1
        td = _torch_dtype(prec)
        dev = nl.pair_offsets.device
        c = torch.empty((N, self.S, self.nmax, self.L2), dtype=td, device=dev)
        dc = dcs = None
        if gradients:
            dc = torch.empty((max(nl.capacity, 1), 3, self.nmax, self.L2), dtype=td, device=dev)
            dcs = torch.empty((N, 3, self.S, self.nmax, self.L2), dtype=td, device=dev)
        vec = _vec_as(nl, td)
        e = self._exec()
        check(self._L.soap_spherical_expansion(self.handle, ctypes.byref(e), prec, N, _ptr(species),
                                               _ptr(nl.pair_offsets), _ptr(nl.pair_j), _ptr(vec), nl.capacity,
                                               _ptr(c), _ptr(dc), _ptr(dcs)))
        return (c, dc, dcs) if gradients else c

    def power_spectrum(self, coeffs: torch.Tensor, precision=None, rows=None, nl: Optional[Neighbors] = None,
                       species: Optional[torch.Tensor] = None):
        """rows = (dc, dcs) gives forward-mode dp rows as well."""
        prec = _precision(precision if precision is not None else coeffs.dtype)
        N = coeffs.shape[0]
        dev = coeffs.device
        td = torch.float64 if prec == SOAP_F64 else torch.float32
        assert coeffs.dtype == td and coeffs.is_contiguous()
        p = torch.empty((N, self.lmax + 1, self.KK), dtype=td, device=dev)
        dp = dps = None
        dc = dcs = None
        if rows is not None:
            dc, dcs = rows
            dp = torch.empty((max(nl.capacity, 1), 3, self.lmax + 1, self.KK), dtype=td, device=dev)
            dps = torch.empty((N, 3, self.lmax + 1, self.KK), dtype=td, device=dev)
        e = self._exec()
        check(self._L.soap_power_spectrum(self.handle, ctypes.byref(e), prec, N, _ptr(coeffs), _ptr(p),
                                          _ptr(species), _ptr(nl.pair_offsets) if nl else None,
                                          _ptr(nl.pair_j) if nl else None, nl.capacity if nl else 0,
                                          _ptr(dc), _ptr(dcs), _ptr(dp), _ptr(dps)))
        return (p, dp, dps) if rows is not None else p

    def features(self, nl: Neighbors, species: torch.Tensor, dtype=torch.float32, gradients=False, out=None,
                 rows: bool = True):
        """soap_features: c and p, with gradients also the self rows and (if
        rows) the pair rows.  out = (c, p[, dc, dcs, dp, dps]) reuses buffers."""
        prec = _precision(dtype)
        td = _torch_dtype(prec)
        N = nl.pair_offsets.shape[0] - 1
        dev = nl.pair_offsets.device
        if out is None:
            out = self.allocate_features(N, nl.capacity, td, dev, gradients)
        c, p = out[0], out[1]
        dc, dcs, dp, dps = (out[2:] if gradients else (None,) * 4)
        if not rows:
            dc = dp = None
        vec = _vec_as(nl, td)
        e = self._exec()
        check(self._L.soap_features(self.handle, ctypes.byref(e), prec, N, _ptr(species), _ptr(nl.pair_offsets),
                                    _ptr(nl.pair_j), _ptr(vec), nl.capacity, _ptr(c), _ptr(p), _ptr(dc),
                                    _ptr(dcs), _ptr(dp), _ptr(dps)))
        return out

    def gradient_rows(self, nl: Neighbors, species: torch.Tensor, coeffs: torch.Tensor, dc=None, dp=None,
                      want_dc=True, want_dp=True):
        """soap_gradient_rows: the pair rows d c / d r_ji and d p / d r_ji."""
        prec = _precision(coeffs.dtype)
        td = coeffs.dtype
        N = nl.pair_offsets.shape[0] - 1
        dev = coeffs.device
        if want_dc and dc is None:
            dc = torch.empty((max(nl.capacity, 1), 3, self.nmax, self.L2), dtype=td, device=dev)
        if want_dp and dp is None:
            dp = torch.empty((max(nl.capacity, 1), 3, self.lmax + 1, self.KK), dtype=td, device=dev)
        vec = _vec_as(nl, td)
        e = self._exec()
        check(self._L.soap_gradient_rows(self.handle, ctypes.byref(e), prec, N, _ptr(species), _ptr(nl.pair_offsets),
                                         _ptr(nl.pair_j), _ptr(vec), nl.capacity, _ptr(coeffs),
                                         _ptr(dc) if want_dc else None, _ptr(dp) if want_dp else None))
        return dc, dp

    def allocate_features(self, N, capacity, td, dev, gradients):
        c = torch.empty((N, self.S, self.nmax, self.L2), dtype=td, device=dev)
        p = torch.empty((N, self.lmax + 1, self.KK), dtype=td, device=dev)
        if not gradients:
            return (c, p)
        dc = torch.empty((max(capacity, 1), 3, self.nmax, self.L2), dtype=td, device=dev)
        dcs = torch.empty((N, 3, self.S, self.nmax, self.L2), dtype=td, device=dev)
        dp = torch.empty((max(capacity, 1), 3, self.lmax + 1, self.KK), dtype=td, device=dev)
        dps = torch.empty((N, 3, self.lmax + 1, self.KK), dtype=td, device=dev)
        return (c, p, dc, dcs, dp, dps)

    def virial(self, nl: Neighbors, grad_pair_vec: torch.Tensor, atom_offsets) -> torch.Tensor:
        """soap_virial: [S, 3, 3], W_s[a][b] = sum over the pairs of the centres
        of structure s of grad_pair_vec[q, a] * pair_vec[q, b]."""
        td = grad_pair_vec.dtype
        prec = _precision(td)
        vec = _vec_as(nl, td)
        dev = grad_pair_vec.device
        ao = torch.as_tensor(np.asarray(atom_offsets, dtype=np.int64) if not isinstance(atom_offsets, torch.Tensor)
                             else atom_offsets, dtype=torch.int64).to(dev).contiguous()
        S = int(ao.shape[0]) - 1
        N = nl.pair_offsets.shape[0] - 1
        part = torch.empty((max(N, 1), 9), dtype=td, device=dev)
        out = torch.empty((max(S, 1), 3, 3), dtype=td, device=dev)
        e = self._exec()
        check(self._L.soap_virial(ctypes.byref(e), prec, S, _ptr(ao), N, _ptr(nl.pair_offsets), _ptr(vec),
                                  _ptr(grad_pair_vec), nl.capacity, _ptr(part), _ptr(out)))
        return out[:S]

    def power_spectrum_selected(self, coeffs: torch.Tensor, selected) -> torch.Tensor:
        """soap_power_spectrum_selected: [N, n_sel] invariants for the
        (k1, k2, l) triples ``selected`` ([n_sel, 3]; see
        ``selection.packed_to_triples``) from coefficients [N, S, nmax, L2]."""
        td = coeffs.dtype
        prec = _precision(td)
        N = coeffs.shape[0]
        c = coeffs.contiguous()
        sel = torch.as_tensor(np.asarray(selected, dtype=np.int32) if not isinstance(selected, torch.Tensor)
                              else selected, dtype=torch.int32).to(c.device).contiguous()
        n_sel = sel.shape[0]
        out = torch.empty((max(N, 1), max(n_sel, 1)), dtype=td, device=c.device)
        e = self._exec()
        check(self._L.soap_power_spectrum_selected(ctypes.byref(e), prec, N, self.K, self.lmax,
                                                   _ptr(c), n_sel, _ptr(sel), _ptr(out)))
        return out[:N, :n_sel]

    def power_spectrum_selected_backward(self, coeffs: torch.Tensor, selected, grad_p: torch.Tensor) -> torch.Tensor:
        """soap_power_spectrum_selected_backward: dL/dc [N, S, nmax, L2] for
        grad_p = dL/dp_sel [N, n_sel]; the plan is built on the host from
        ``selected`` and copied to the device."""
        td = coeffs.dtype
        prec = _precision(td)
        N = coeffs.shape[0]
        c = coeffs.contiguous()
        tri = np.ascontiguousarray(selected.cpu().numpy() if isinstance(selected, torch.Tensor) else selected,
                                   dtype=np.int32).reshape(-1, 3)
        n_sel = tri.shape[0]
        offs = np.zeros(self.K * (self.lmax + 1) + 1, dtype=np.int32)
        ent = np.zeros((max(2 * n_sel, 1), 2), dtype=np.int32)
        check(self._L.soap_power_spectrum_selected_plan(self.K, self.lmax, n_sel, _np_ptr(tri), _np_ptr(offs),
                                                        _np_ptr(ent)))
        offs_d = torch.from_numpy(offs).to(c.device)
        ent_d = torch.from_numpy(ent).to(c.device)
        g = grad_p.to(td).contiguous()
        gc = torch.empty_like(c)
        e = self._exec()
        check(self._L.soap_power_spectrum_selected_backward(ctypes.byref(e), prec, N, self.K, self.lmax, _ptr(c), n_sel,
                                                            _ptr(g), _ptr(offs_d), _ptr(ent_d), _ptr(gc)))
        return gc

    def gpr_predict(self, species: torch.Tensor, features: torch.Tensor, active_species: torch.Tensor,
                    active_features: torch.Tensor, weights: torch.Tensor, zeta: int, want_grad: bool = True):
        """soap_gpr_predict: per-centre energies [N] of the sparse kernel model
        and, if want_grad, dE/dp [N, F] (None otherwise); features [N, ...]
        are flattened per centre."""
        td = features.dtype
        prec = _precision(td)
        N = features.shape[0]
        p = features.reshape(N, -1).contiguous()
        F = p.shape[1]
        M = active_features.reshape(active_features.shape[0], -1).to(td).contiguous()
        if M.shape[1] != F:
            raise ValueError(f"active_features have {M.shape[1]} features per point, features {F}")
        nA = M.shape[0]
        w = weights.to(td).contiguous()
        sp = species.to(torch.int32).contiguous()
        asp = active_species.to(device=p.device, dtype=torch.int32).contiguous()
        if w.shape[0] != nA or asp.shape[0] != nA or sp.shape[0] != N:
            raise ValueError("species, active_species and weights must match the feature rows")
        nb = ctypes.c_size_t()
        check(self._L.soap_gpr_workspace_size(prec, N, F, nA, ctypes.byref(nb)))
        ws = torch.empty(max(nb.value // p.element_size(), 1), dtype=td, device=p.device)
        energies = torch.empty(max(N, 1), dtype=td, device=p.device)
        grad = torch.empty((max(N, 1), F), dtype=td, device=p.device) if want_grad else None
        e = self._exec()
        check(self._L.soap_gpr_predict(ctypes.byref(e), prec, N, F, _ptr(sp), _ptr(p), nA, _ptr(asp), _ptr(M),
                                       _ptr(w), int(zeta), _ptr(ws), nb.value, _ptr(energies), _ptr(grad)))
        return energies[:N], (grad[:N] if want_grad else None)

    def power_spectrum_backward(self, coeffs: torch.Tensor, grad_p: torch.Tensor) -> torch.Tensor:
        prec = _precision(coeffs.dtype)
        N = coeffs.shape[0]
        grad_p = grad_p.contiguous().to(coeffs.dtype)
        gc = torch.empty_like(coeffs)
        e = self._exec()
        check(self._L.soap_power_spectrum_backward(self.handle, ctypes.byref(e), prec, N, _ptr(coeffs),
                                                   _ptr(grad_p), _ptr(gc)))
        return gc

    def spherical_expansion_backward(self, nl: Neighbors, species: torch.Tensor, grad_coeffs: torch.Tensor):
        prec = _precision(grad_coeffs.dtype)
        td = grad_coeffs.dtype
        N = nl.pair_offsets.shape[0] - 1
        dev = grad_coeffs.device
        grad_coeffs = grad_coeffs.contiguous()
        gpair = torch.empty((max(nl.capacity, 1), 3), dtype=td, device=dev)
        gpos = torch.empty((N, 3), dtype=td, device=dev)
        vec = _vec_as(nl, td)
        e = self._exec()
        check(self._L.soap_spherical_expansion_backward(self.handle, ctypes.byref(e), prec, N, _ptr(species),
                                                        _ptr(nl.pair_offsets), _ptr(nl.pair_j), _ptr(vec),
                                                        _ptr(nl.pair_transpose), nl.capacity, _ptr(grad_coeffs),
                                                        _ptr(gpair), _ptr(gpos)))
        return gpos, gpair


def _vec_as(nl: Neighbors, td) -> torch.Tensor:
    if nl.pair_vec.dtype != td:
        raise ValueError(f"pair_vec is {nl.pair_vec.dtype}, the call needs {td}: build the list with vec_dtype={td}")
    return nl.pair_vec


def structures_to_device(atom_offsets, cells, pbc, device):
    """(atom_offsets int64 [S+1], cells float64 [S,3,3], pbc uint8 [S,3]) on the device."""
    def conv(x, dtype, shape):
        if isinstance(x, torch.Tensor) and x.is_cuda:
            assert x.dtype == dtype and x.is_contiguous()
            return x
        a = np.ascontiguousarray(np.asarray(x.cpu() if isinstance(x, torch.Tensor) else x))
        return torch.tensor(a.reshape(shape), dtype=dtype, device=device)
    ao = conv(atom_offsets, torch.int64, (-1,))
    n = int(ao.shape[0] - 1)
    return ao, conv(cells, torch.float64, (n, 3, 3)), conv(pbc, torch.uint8, (n, 3))


class SOAPFunction(torch.autograd.Function):
    """positions -> power spectrum, differentiable with respect to positions
    through the hand-written adjoint kernels (soap_power_spectrum_backward
    followed by soap_spherical_expansion_backward).  The neighbour list is
    built once per forward call and reused by the backward call.

    Both passes read the device status word before returning (one
    synchronisation each) and raise SoapError if a kernel reported an error:
    a coincident pair, an invalid species or a pair without its reverse
    would otherwise give wrong features or forces silently."""

    @staticmethod
    def forward(ctx, positions, calc: Calculator, species, atom_offsets, cells, pbc, dtype=torch.float32):
        nl = calc.compute_neighbors(positions.detach(), species, atom_offsets, cells, pbc, vec_dtype=dtype)
        c, p = calc.features(nl, species, dtype=dtype)
        calc.check_device()
        ctx.calc, ctx.nl, ctx.species = calc, nl, species
        ctx.save_for_backward(c)
        return p

    @staticmethod
    def backward(ctx, grad_p):
        (c,) = ctx.saved_tensors
        gc = ctx.calc.power_spectrum_backward(c, grad_p.to(c.dtype))
        gpos, _ = ctx.calc.spherical_expansion_backward(ctx.nl, ctx.species, gc)
        ctx.calc.check_device()
        return gpos.to(torch.float64), None, None, None, None, None, None


def soap_power_spectrum_of_positions(positions, calc, species, atom_offsets, cells, pbc, dtype=torch.float32):
    return SOAPFunction.apply(positions, calc, species, atom_offsets, cells, pbc, dtype)


class Compressor:
    """The learned equivariant channel compression of a calculator's
    coefficients (soap_compress_*, soap_spectrum_*, soap_adam_step): per l a
    two-layer network on the (species, n) channels, shared over m, with a
    norm gate.  Holds the weights and the Adam moments on the device."""

    def __init__(self, calc: Calculator, n_out: int = 16, hidden: int = 128, device=None):
        self.calc, self.Q, self.H = calc, int(n_out), int(hidden)
        L = calc._L
        n = ctypes.c_int64()
        check(L.soap_compress_n_params(calc.handle, self.Q, self.H, ctypes.byref(n)))
        ws = ctypes.c_size_t()
        check(L.soap_compress_workspace_size(calc.handle, self.Q, self.H, ctypes.byref(ws)))
        dev = device if device is not None else torch.device("cuda", torch.cuda.current_device())
        self.n_params = int(n.value)
        self.weights = torch.zeros(self.n_params, dtype=torch.float32, device=dev)
        self._ws = torch.empty(max(int(ws.value), 256), dtype=torch.uint8, device=dev)
        self._m = torch.zeros_like(self.weights)
        self._v = torch.zeros_like(self.weights)
        self._grad = torch.zeros_like(self.weights)
        self._loss = torch.zeros(1, dtype=torch.float32, device=dev)
        self.step = 0

    @property
    def lmax(self) -> int:
        return self.calc.lmax

    def init_pca(self, coeffs: torch.Tensor, seed: int = 0, noise: float = 0.1):
        """soap_compress_init_pca over the centres of coeffs [N, S, nmax, L2] (float)."""
        assert coeffs.dtype == torch.float32 and coeffs.is_contiguous()
        e = self.calc._exec()
        check(self.calc._L.soap_compress_init_pca(self.calc.handle, ctypes.byref(e), self.Q, self.H,
                                                  int(coeffs.shape[0]), _ptr(coeffs), ctypes.c_uint64(seed),
                                                  float(noise), _ptr(self._ws), self._ws.numel(),
                                                  _ptr(self.weights)))
        self._m.zero_()
        self._v.zero_()
        self.step = 0

    def forward(self, coeffs: torch.Tensor, precision=torch.float32, want_coeffs: bool = False, want_p: bool = True):
        """soap_compress_forward: (c~ [N, Q, L2] or None, p~ [N, lmax+1, Q(Q+1)/2] or None)."""
        assert coeffs.dtype == torch.float32 and coeffs.is_contiguous()
        N, dev = int(coeffs.shape[0]), coeffs.device
        prec = SOAP_BF16_F32ACC if precision in ("bf16", torch.bfloat16, SOAP_BF16_F32ACC) else SOAP_F32
        ct = torch.empty((N, self.Q, self.calc.L2), dtype=torch.float32, device=dev) if want_coeffs else None
        pt = (torch.empty((N, self.lmax + 1, self.Q * (self.Q + 1) // 2), dtype=torch.float32, device=dev)
              if want_p else None)
        e = self.calc._exec()
        if prec == SOAP_BF16_F32ACC and self._ws.device == dev:
            # the weights laid out once in the workspace (bit for bit the
            # same results as soap_compress_forward)
            check(self.calc._L.soap_compress_forward_ws(self.calc.handle, ctypes.byref(e), prec, self.Q, self.H, N,
                                                        _ptr(self.weights), _ptr(coeffs), _ptr(ct), _ptr(pt),
                                                        _ptr(self._ws), self._ws.numel()))
        else:
            check(self.calc._L.soap_compress_forward(self.calc.handle, ctypes.byref(e), prec, self.Q, self.H, N,
                                                     _ptr(self.weights), _ptr(coeffs), _ptr(ct), _ptr(pt)))
        return ct, pt

    def forward_plain(self, coeffs: torch.Tensor, precision=torch.float32, want_coeffs: bool = False,
                      want_p: bool = True):
        """soap_compress_forward without a workspace (the weights staged from
        their float form for every degree)."""
        N, dev = int(coeffs.shape[0]), coeffs.device
        prec = SOAP_BF16_F32ACC if precision in ("bf16", torch.bfloat16, SOAP_BF16_F32ACC) else SOAP_F32
        ct = torch.empty((N, self.Q, self.calc.L2), dtype=torch.float32, device=dev) if want_coeffs else None
        pt = (torch.empty((N, self.lmax + 1, self.Q * (self.Q + 1) // 2), dtype=torch.float32, device=dev)
              if want_p else None)
        e = self.calc._exec()
        check(self.calc._L.soap_compress_forward(self.calc.handle, ctypes.byref(e), prec, self.Q, self.H, N,
                                                 _ptr(self.weights), _ptr(coeffs), _ptr(ct), _ptr(pt)))
        return ct, pt

    def backward(self, coeffs: torch.Tensor, grad_p: torch.Tensor, out: Optional[torch.Tensor] = None):
        """soap_compress_backward: dL/dweights for dL/dp~ = grad_p."""
        assert grad_p.dtype == torch.float32 and grad_p.is_contiguous()
        out = self._grad if out is None else out
        e = self.calc._exec()
        check(self.calc._L.soap_compress_backward(self.calc.handle, ctypes.byref(e), self.Q, self.H,
                                                  int(coeffs.shape[0]), _ptr(self.weights), _ptr(coeffs),
                                                  _ptr(grad_p), _ptr(self._ws), self._ws.numel(), _ptr(out)))
        return out

    def gram(self, X: torch.Tensor, n_channels: int) -> torch.Tensor:
        """soap_spectrum_gram of packed spectra X [n, lmax+1, Q(Q+1)/2]."""
        assert X.dtype == torch.float32 and X.is_contiguous()
        n = int(X.shape[0])
        K = torch.empty((n, n), dtype=torch.float32, device=X.device)
        e = self.calc._exec()
        check(self.calc._L.soap_spectrum_gram(ctypes.byref(e), n, int(n_channels), self.lmax, _ptr(X), _ptr(K)))
        return K

    def kernel_loss(self, X: torch.Tensor, Kref: torch.Tensor):
        """soap_spectrum_kernel_loss for compressed spectra X: (loss as a
        device tensor [1], dL/dX)."""
        n = int(X.shape[0])
        work = torch.empty(n * n + 1, dtype=torch.float32, device=X.device)
        gX = torch.empty_like(X)
        e = self.calc._exec()
        check(self.calc._L.soap_spectrum_kernel_loss(ctypes.byref(e), n, self.Q, self.lmax, _ptr(X), _ptr(Kref),
                                                     _ptr(work), _ptr(self._loss), _ptr(gX)))
        return self._loss, gX

    def adam(self, lr: float, beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8):
        """soap_adam_step on the weights with the last gradient."""
        self.step += 1
        e = self.calc._exec()
        check(self.calc._L.soap_adam_step(ctypes.byref(e), self.n_params, _ptr(self.weights), _ptr(self._grad),
                                          _ptr(self._m), _ptr(self._v), float(lr), float(beta1), float(beta2),
                                          float(eps), self.step))

    def train_step(self, coeffs: torch.Tensor, lr: float) -> torch.Tensor:
        """One Adam step on a batch of centres: full spectrum and its kernel
        (the reference), compressed spectrum, loss, gradients.  Returns the
        loss before the step (device tensor)."""
        pf = self.calc.power_spectrum(coeffs, precision=torch.float32)
        Kref = self.gram(pf.reshape(pf.shape[0], self.lmax + 1, -1), self.calc.K)
        _, pt = self.forward(coeffs)
        loss, gX = self.kernel_loss(pt, Kref)
        loss = loss.clone()
        self.backward(coeffs, gX)
        self.adam(lr)
        return loss

    def save(self, path: str) -> None:
        """soap_compress_save: the weights, the Adam moments and step, with the
        shape (n_out, hidden, channels, lmax) and a hash, to a binary file."""
        check(self.calc._L.soap_compress_save(self.calc.handle, self.Q, self.H, int(self.step), _ptr(self.weights),
                                              _ptr(self._m), _ptr(self._v), os.fsencode(path)))

    def load(self, path: str) -> None:
        """soap_compress_load: reads a file written by save(); SoapError
        (SOAP_EINVAL) if its shape differs from this compressor's, or it is
        truncated or corrupted."""
        step = ctypes.c_int64()
        check(self.calc._L.soap_compress_load(self.calc.handle, self.Q, self.H, os.fsencode(path), _ptr(self.weights),
                                              _ptr(self._m), _ptr(self._v), ctypes.byref(step)))
        self.step = int(step.value)

    def kernel_error(self, coeffs: torch.Tensor, precision=torch.float32) -> float:
        """eps_K = |K~ - K|_F / |K|_F over the centres of coeffs (synchronises)."""
        pf = self.calc.power_spectrum(coeffs, precision=torch.float32)
        Kref = self.gram(pf.reshape(pf.shape[0], self.lmax + 1, -1), self.calc.K)
        _, pt = self.forward(coeffs, precision=precision)
        loss, _ = self.kernel_loss(pt, Kref)
        return float(loss.item()) ** 0.5
