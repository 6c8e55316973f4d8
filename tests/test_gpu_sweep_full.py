"""The order-sweep workload at full size: N = 1..15, about 2^24 local nodes each,
jittered, in the launch configuration the sweep measures (default tile
schedules).  Every output of the FP64 operator is compared with the oracle
(1e-12 relative), and the FP32 operator with the same derived bar as the
small cases (parity unpinned: no FP32 reference exists); the two-phase operator
(HB_MESH_GATHER) on the same mesh and input to the FP64 bar."""
import sys

import numpy as np
import pytest

import inputs
import oracle

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2202_12477_amd as hb  # noqa: E402


def relerr(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


@pytest.mark.parametrize("N", list(range(1, 16)))
def test_order_sweep_full_size(N):
    c = inputs.order_sweep_case(N)
    print(f"[case] order sweep N={N} n={c.nx} full size", flush=True)
    sys.stdout.flush()
    ref = oracle.Mesh(c.nx, c.ny, c.nz, c.N, jitter=c.jitter, seed=c.mesh_seed)
    x = inputs.random_vector(ref.NG, 200 + N)
    yref = ref.ax(x, c.lam)
    del ref
    m = hb.Mesh(c.nx, c.ny, c.nz, c.N, jitter=c.jitter, seed=c.mesh_seed, fp32=True)
    assert m.NL >= 16_000_000
    xd = torch.as_tensor(x, device="cuda")
    y = torch.empty_like(xd)
    m.ax(c.lam, xd, y)
    y32 = torch.empty(m.NG, dtype=torch.float32, device="cuda")
    m.ax_f32(c.lam, xd, y32)
    torch.cuda.synchronize()
    e64 = relerr(y.cpu().numpy(), yref)
    e32 = relerr(y32.cpu().numpy().astype(np.float64), yref)
    m.close()
    del y32
    g = hb.Mesh(c.nx, c.ny, c.nz, c.N, jitter=c.jitter, seed=c.mesh_seed, gather=True)
    yg = torch.empty_like(xd)
    g.ax(c.lam, xd, yg)
    torch.cuda.synchronize()
    eg = relerr(yg.cpu().numpy(), yref)
    g.close()
    print(f"N={N}: FP64 {e64:.2e}, FP32 {e32:.2e}, two-phase {eg:.2e}", flush=True)
    assert e64 <= 1e-12 and eg <= 1e-12
    assert 1e-9 < e32 <= 2e-5
