"""soap_compute_neighbors_noalloc (static device scratch, no allocation)
against soap_compute_neighbors with a caller workspace, through the C ABI.

Both entry points run the same kernels, so every output (CSR offsets, pair
indices, shifts, vectors, reverse-pair index) must agree bit for bit; two
calls in a row, the second on a smaller input, check that the scratch left
by the first call does not leak into the second."""
import ctypes

import pytest
import torch

import synthetic
import paper_2101_08814_amd as P
from paper_2101_08814_amd import _lib
from paper_2101_08814_amd.soap import structures_to_device

pytestmark = pytest.mark.gpu


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _outputs(N, cap, vec_dtype, dev):
    return (torch.full((N + 1,), -7, dtype=torch.int64, device=dev),
            torch.full((cap,), -7, dtype=torch.int32, device=dev),
            torch.full((cap, 3), -7, dtype=torch.int32, device=dev),
            torch.full((cap, 3), -7.0, dtype=vec_dtype, device=dev),
            torch.full((cap,), -7, dtype=torch.int32, device=dev))


def _run_both(batch, vec_dtype):
    dev = torch.device("cuda", 0)
    L = _lib.lib()
    calc = P.Calculator.from_hypers(batch.hypers)
    pos = torch.tensor(batch.positions, dtype=torch.float64, device=dev)
    spc = torch.tensor(batch.species, dtype=torch.int32, device=dev)
    ao, ce, pb = structures_to_device(batch.atom_offsets, batch.cells, batch.pbc, dev)
    N, n_struct = batch.n_atoms, batch.n_structures
    cap = calc.compute_neighbors(pos, spc, ao, ce, pb, vec_dtype=vec_dtype).count() + 5
    prec = _lib.SOAP_F64 if vec_dtype == torch.float64 else _lib.SOAP_F32
    status = torch.zeros(1, dtype=torch.int32, device=dev)
    ex = _lib.soap_exec(ctypes.c_void_p(torch.cuda.current_stream().cuda_stream), ctypes.c_void_p(status.data_ptr()))
    ws_n = ctypes.c_size_t()
    _lib.check(L.soap_neighbors_workspace_size(calc.handle, n_struct, N, ctypes.byref(ws_n)))
    ws = torch.empty(max(ws_n.value, 256), dtype=torch.uint8, device=dev)
    ref = _outputs(N, cap, vec_dtype, dev)
    _lib.check(L.soap_compute_neighbors(calc.handle, ctypes.byref(ex), n_struct, N, _ptr(ao), _ptr(ce), _ptr(pb),
                                        _ptr(pos), _ptr(spc), _ptr(ws), ws.numel(), cap, prec,
                                        *[_ptr(t) for t in ref]))
    got = _outputs(N, cap, vec_dtype, dev)
    _lib.check(L.soap_compute_neighbors_noalloc(calc.handle, ctypes.byref(ex), n_struct, N, _ptr(ao), _ptr(ce),
                                                _ptr(pb), _ptr(pos), _ptr(spc), cap, prec,
                                                *[_ptr(t) for t in got]))
    assert int(L.soap_read_device_status(ctypes.byref(ex))) == 0
    n_pairs = int(ref[0][-1].item())
    assert n_pairs > 0 and n_pairs <= cap
    for name, a, b in zip(("pair_offsets", "pair_j", "pair_shift", "pair_vec", "pair_transpose"), ref, got):
        assert torch.equal(a, b), f"{name} differs between the workspace and no-allocation entry points"
    return N, n_pairs


@pytest.mark.parametrize("vec_dtype", [torch.float32, torch.float64])
def test_noalloc_neighbors_two_calls(vec_dtype):
    print(f"[no-alloc] diamond 1024 then clusters 128, {vec_dtype}", flush=True)
    n1, p1 = _run_both(synthetic.diamond_bulk(), vec_dtype)
    n2, p2 = _run_both(synthetic.clusters_2species().subset([0, 1]), vec_dtype)
    assert n2 < n1 and p2 < p1


def test_noalloc_neighbors_many_structures():
    """The multi-launch bin build (more than 8192 atoms): 64 of the
    8-species cells, then a smaller batch of 8."""
    print("[no-alloc] 64 then 8 periodic 8-species cells", flush=True)
    big = synthetic.multi_species_cells(n_cells=64)
    n1, p1 = _run_both(big, torch.float32)
    n2, p2 = _run_both(big.subset(list(range(8))), torch.float32)
    assert n2 < n1 and p2 < p1


def test_noalloc_rejects_oversized_request():
    L = _lib.lib()
    calc = P.Calculator(1, 2, 1, 3.0, 0.5)
    dummy = torch.zeros(64, dtype=torch.float64, device="cuda")
    ex = _lib.soap_exec(None, None)
    p = _ptr(dummy)
    st = L.soap_compute_neighbors_noalloc(calc.handle, ctypes.byref(ex), 1, 1 << 20, p, p, p, p, p, 16,
                                          _lib.SOAP_F32, p, p, p, p, None)
    assert st == _lib.SOAP_EINVAL
    assert b"static scratch" in L.soap_last_error()
