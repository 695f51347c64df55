"""GPU: the allocation-free surrogate entry point pamd_nn_forces_static
against pamd_nn_forces (through the C ABI).  Both run the same kernels on the
same inputs, so energies and forces must agree bit for bit; two calls in a
row, the second with a smaller batch, show that nothing left in the shared
staging array from the first call leaks into the second.  A batch beyond the
fixed staging is refused."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from pamd_inputs import systems as S  # noqa: E402
from pamd_inputs.weights import surrogate_weights  # noqa: E402


@pytest.fixture(scope="module")
def B():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1806_06016_amd import pamd
    pamd.load_library()
    return pamd


def test_static_forces_equal_workspace_forces(B):
    sysd = S.c2_system()
    n = sysd.n_atoms
    big = B.NN_STATIC_ROWS // n            # 213 configurations: the largest batch the staging takes
    nn = B.PamdNN(sysd, sysd.atype, max_conf=big)
    nn.set_weights(surrogate_weights(3))
    for nb, seed in ((big, 1), (37, 2)):
        print("static surrogate forces, batch", nb, flush=True)
        rng = np.random.default_rng(seed)
        x = torch.tensor(sysd.x_init[None] + rng.normal(0, 0.02, (nb,) + sysd.x_init.shape), dtype=torch.float32,
                         device="cuda")
        E1, F1 = nn.forces(x)
        E2, F2 = nn.forces_static(x)
        torch.cuda.synchronize()
        assert torch.isfinite(F1).all() and torch.count_nonzero(F1).item() > 0
        assert torch.equal(E1, E2) and torch.equal(F1, F2)
    with pytest.raises(B.PamdError) as ei:
        x = torch.zeros((big + 1, n, 3), dtype=torch.float32, device="cuda")
        nn.forces_static(x)
    assert ei.value.code == B.PAMD_ERR_ARG and "PAMD_NN_STATIC_ROWS" in str(ei.value)
    nn.close()
