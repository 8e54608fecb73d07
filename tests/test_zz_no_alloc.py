"""The allocation-free entry point (qtn_energy_grad_noalloc) against
qtn_energy_grad on the same nets, through the C ABI: two calls in a row, the
second on a smaller network, both forms, plus the size limit of the static
scratch.  Tolerances are those of the oracle comparisons: complex64 energies
within 1e-5 relative, per-edge <ZZ> within 1e-5 absolute, gradients within
1e-4 of their largest component; complex128 within 1e-10.
"""
import numpy as np
import pytest

from workloads import workload

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _net(name, **kw):
    from paper_2106_15740_amd import QaoaNet

    w = workload(name)
    print(f"[case] {name} n={w.n} m={len(w.edges)} p={w.p} {kw}", flush=True)
    net = QaoaNet(w.n, w.edges, w.p, dtype=kw.get("dtype", w.dtype), order=w.order, device=0)
    net.set_params(w.gamma, w.beta)
    return net


def _compare(net, mode, tol):
    zz_a = net.zz_buffer()
    e_a, dg_a, db_a = net.energy_grad_noalloc(mode, zz_out=zz_a)
    z_res, dz_res = net.edge_results(with_grad=True)  # NULL workspace: the scratch of that call
    zz_b = net.zz_buffer()
    e_b, dg_b, db_b = net.energy_grad(mode, zz_out=zz_b)
    z_ref, dz_ref = net.edge_results(with_grad=True)
    assert abs(e_a - e_b) <= tol * abs(e_b), (mode, e_a, e_b)
    gs = max(np.abs(dg_b).max(), np.abs(db_b).max(), 1e-300)
    grad_tol = 1e-4 if tol > 1e-8 else 1e-9
    np.testing.assert_allclose(dg_a, dg_b, rtol=0, atol=grad_tol * gs)
    np.testing.assert_allclose(db_a, db_b, rtol=0, atol=grad_tol * gs)
    np.testing.assert_allclose(zz_a.cpu().numpy(), zz_b.cpu().numpy(), rtol=0, atol=tol)
    np.testing.assert_allclose(z_res, z_ref, rtol=0, atol=tol)
    ds = max(np.abs(dz_ref).max(), 1e-300)
    np.testing.assert_allclose(dz_res, dz_ref, rtol=0, atol=grad_tol * ds)
    return e_a


@pytest.mark.parametrize("mode", ["batched", "plain"])
def test_noalloc_matches_workspace_entry_point(mode):
    from paper_2106_15740_amd import _lib as L

    big = _net("p3_n244")
    assert big.workspace_size(True) <= L.QTN_SCRATCH_BYTES
    e_big = _compare(big, mode, 1e-5)
    # the second call in a row, on a smaller network: the scratch still holds
    # the first call's contents
    small = _net("p2_n60")
    assert small.workspace_size(True) < big.workspace_size(True)
    e_small = _compare(small, mode, 1e-5)
    assert e_small != e_big
    tiny = _net("p1_n10")
    _compare(tiny, mode, 1e-10)


def test_noalloc_rejects_networks_beyond_the_scratch():
    from paper_2106_15740_amd import _lib as L

    net = _net("p4_n100")
    assert net.workspace_size(True) > L.QTN_SCRATCH_BYTES
    with pytest.raises(L.QtnError) as ei:
        net.energy_grad_noalloc("batched")
    assert ei.value.status == L.QTN_ENOMEM
    # the library is still usable afterwards
    small = _net("p2_n60")
    _compare(small, "batched", 1e-5)
