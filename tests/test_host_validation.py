"""Host-side parameter validation of the C ABI (no GPU call is made):
lbm_workspace_bytes returns 0 and lbm_last_error names the cause for every
parameter set the library rejects, and the workspace size of a valid lattice
holds the two time levels of the 27 populations."""
import ctypes as C

import pytest

from paper_2306_11320_amd import workloads as wl

lbm = pytest.importorskip("paper_2306_11320_amd.lbm")


def _lib():
    try:
        return lbm.lib()
    except RuntimeError as e:
        pytest.fail(str(e))


def _params(**over):
    cfg, _ = wl.tiny(40, 24, bc=wl.ALL_BCS[1], seed=1)
    p = lbm.make_params(cfg, lbm.FP32_DEV)
    for k, v in over.items():
        if k == "bc":
            for s in range(4):
                p.bc[s] = v[s]
        else:
            setattr(p, k, v)
    return p


def test_valid_lattice_workspace():
    L = _lib()
    p = _params()
    n = L.lbm_workspace_bytes(C.byref(p))
    plane = 48 * 24  # FP32 rows start every 16 nodes: 40 -> 48, 18 whole 64-node blocks
    assert n >= 2 * 27 * plane * 4 + 2 * plane * 4
    p64 = _params(precision=lbm.FP64)
    plane64 = 40 * 24  # FP64 rows packed with no gap: 960 nodes, 15 blocks
    assert L.lbm_workspace_bytes(C.byref(p64)) >= 2 * 27 * plane64 * 8 + 2 * plane64 * 8
    # a node count that is not a multiple of the block is rounded up to one
    odd = _params(nx=41, ny=23, precision=lbm.FP64)
    assert L.lbm_workspace_bytes(C.byref(odd)) >= 2 * 27 * 960 * 8 + 2 * 960 * 8


@pytest.mark.parametrize("over,why", [
    (dict(abi_version=lbm.ABI_VERSION + 1), "abi_version"),
    (dict(nx=2), "smaller than 3x3"),
    (dict(nx=20000, ny=20000), "too large"),
    (dict(precision=7), "precision"),
    (dict(bc=[wl.PERIODIC, wl.WALL_T, wl.WALL_T, wl.WALL_T]), "periodic paired"),
    (dict(grad_mode=2), "grad_mode"),
    (dict(collision=2), "collision"),
    (dict(force_form=2), "force_form"),
    (dict(collision=lbm.TRT, trt_magic=0.0), "trt_magic"),
    (dict(n_bubbles=5), "tracked regions"),
    (dict(rho_l=0.0), "densities"),
    (dict(mu_h=-1.0), "viscosities"),
    (dict(lambda_l=0.0), "conductivities"),
    (dict(rhocp_h=0.0), "heat capacitances"),
    (dict(mobility=0.0), "mobility"),
    (dict(W=0.0), "interface width"),
])
def test_rejected_parameters(over, why):
    L = _lib()
    p = _params(**over)
    assert L.lbm_workspace_bytes(C.byref(p)) == 0
    assert why in L.lbm_last_error().decode()


@pytest.mark.parametrize("prec,word", [(lbm.FP32_DEV, 4), (lbm.FP64, 8)])
def test_lattice_size_limit(prec, word):
    """One time level (nx, rounded up to 16 in FP32, times ny, rounded up to
    64, times 27 values) must stay below 4 GiB: the kernels address a level
    with 32-bit byte offsets."""
    L = _lib()
    nx = 4096
    ny_max = (2 ** 32 - 1) // (nx * 27 * word)
    ok = _params(precision=prec, nx=nx, ny=ny_max)
    assert L.lbm_workspace_bytes(C.byref(ok)) >= 2 * 27 * nx * ny_max * word
    bad = _params(precision=prec, nx=nx, ny=ny_max + 1)
    assert L.lbm_workspace_bytes(C.byref(bad)) == 0
    assert "4 GiB" in L.lbm_last_error().decode()


@pytest.mark.parametrize("nx", [2 ** 32 - 10, 2 ** 31])
def test_huge_width_rejected(nx):
    """Widths near 2^32 (which would wrap when rounded up to whole 64-node
    blocks in 32-bit arithmetic) and widths beyond a signed 32-bit integer are
    rejected, not accepted as a small lattice."""
    L = _lib()
    p = _params(nx=nx, ny=3)
    assert L.lbm_workspace_bytes(C.byref(p)) == 0
    assert "signed 32-bit" in L.lbm_last_error().decode()


def test_heat_capacitance_below_one_warns():
    """rho c_p < 1 is accepted (the blend of Eq. 28 is then not a convex
    combination): the workspace is sized and the message text holds a warning."""
    L = _lib()
    ok = _params(rhocp_l=1.0, rhocp_h=2.0)
    assert L.lbm_workspace_bytes(C.byref(ok)) > 0
    p = _params(rhocp_l=0.5, rhocp_h=2.0)
    assert L.lbm_workspace_bytes(C.byref(p)) > 0
    msg = L.lbm_last_error().decode()
    assert msg.startswith("warning:") and "heat capacitance" in msg
