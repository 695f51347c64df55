"""GPU: properties the paper's MD relies on, measured on the GPU path itself
(through the C ABI), and the error paths of the optional calls.

* NVE (nu = 0) energy error of velocity Verlet shrinks as dt^2: RMS of
  E_tot(t) - E_tot(0) over a fixed window at three time steps, log-log slope
  in [1.8, 2.2] (bead chain, FP64) and [1.7, 2.3] (peptide, FP32 positions).
* Total momentum is conserved by NVE dynamics (FP64 bead chain: 1e-12
  relative to sum |m v|).
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from oracle import oracle as O  # noqa: E402
from pamd_inputs import systems as S  # noqa: E402


@pytest.fixture(scope="module")
def B():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1806_06016_amd import pamd
    pamd.load_library()
    return pamd


def _drift(B, sysd, x, v, T, dt, window, samples, prec):
    p = B.Pamd([sysd], R_target=x.shape[0], T0=T, dt=dt, nu=0.0, seed=5, precision=prec)
    p.set_state(0, x, v, T=T)
    p.md_steps(0)
    st = p.get_state(0, want_xv=False)
    E0 = st["E_pot"] + st["E_kin"]
    k = int(round(window / samples / dt))
    dev = []
    for _ in range(samples):
        p.md_steps(k)
        st = p.get_state(0, want_xv=False)
        dev.append(st["E_pot"] + st["E_kin"] - E0)
    p.close()
    return float(np.sqrt(np.mean(np.square(dev))))


def _thermalised(sysd, R, T, dt, steps, seed):
    osys = O.OracleSystem(sysd)
    x = np.ascontiguousarray(np.broadcast_to(sysd.x_init, (R, sysd.n_atoms, 3)).astype(np.float64))
    v = O.init_velocities(osys, R, T, seed=seed)
    O.md_steps(osys, x, v, steps, T, dt, 1.0, seed, 0)
    return x, v


@pytest.mark.parametrize("which", ["chain", "peptide"])
def test_nve_energy_error_scales_as_dt_squared(B, which):
    if which == "chain":
        sysd, T, prec, dts, window, lo, hi = S.c1_system(), 1.0, 0, [0.004, 0.002, 0.001], 4.0, 1.8, 2.2
        x, v = _thermalised(sysd, 64, T, 0.002, 1000, 9)
    else:
        sysd, T, prec, dts, window, lo, hi = S.c2_system(), 300.0, 1, [0.001, 0.0005, 0.00025], 1.0, 1.7, 2.3
        x, v = _thermalised(sysd, 64, T, 0.0005, 4000, 9)
    print(f"NVE drift {which}", flush=True)
    errs = [_drift(B, sysd, x, v, T, dt, window, 20, prec) for dt in dts]
    slope = np.polyfit(np.log(dts), np.log(errs), 1)[0]
    print("errors", errs, "slope", slope)
    assert lo <= slope <= hi


def test_nve_conserves_momentum(B):
    sysd = S.c1_system()
    x, v = _thermalised(sysd, 32, 1.0, 0.002, 200, 4)
    p = B.Pamd([sysd], R_target=32, T0=1.0, dt=0.002, nu=0.0, seed=5, precision=0)
    p.set_state(0, x, v, T=1.0)
    m = sysd.mass[None, :, None]
    P0 = (m * p.get_state(0)["v"]).sum(1)
    p.md_steps(1000)
    g = p.get_state(0)
    P1 = (m * g["v"]).sum(1)
    scale = (m * np.abs(g["v"])).sum(1)
    assert np.all(np.abs(P1 - P0) <= 1e-12 * scale)
    p.close()


def test_resample_before_md_is_a_state_error(B):
    sysd = S.c1_system()
    p = B.Pamd([sysd], R_target=16, T0=2.0, dt=0.002, nu=1.0, seed=1, precision=0)
    with pytest.raises(B.PamdError) as e:
        p.resample([1.9])
    assert e.value.code == B.PAMD_ERR_STATE
    p.md_steps(0)                              # energies now exist
    p.resample([1.9])
    assert p.observables()[0]["T"] == 1.9
    p.close()


def test_optional_call_errors(B):
    """r-RESPA needs an FP32 context of molecules within the register tiles, a
    step count that is a multiple of the outer ratio; export likewise."""
    sysd = S.c2_system()
    nn = B.PamdNN(sysd, sysd.atype)
    p = B.Pamd([sysd], R_target=16, T0=700.0, dt=0.001, nu=1.0, seed=1, precision=B.PAMD_FP32)
    p.set_mts(nn, 4)
    with pytest.raises(B.PamdError) as e:
        p.md_steps(6)
    assert e.value.code == B.PAMD_ERR_ARG
    p.md_steps(8)                              # a multiple of 4 runs
    p.md_steps(0)                              # energies only
    p.set_mts(None)
    p.md_steps(3)                              # plain MD again
    p.close()
    wide = B.Pamd([S.make_peptide(1806, 120)], R_target=16, T0=700.0, dt=0.0005, nu=1.0, seed=1,
                  precision=B.PAMD_FP32)
    with pytest.raises(B.PamdError):
        wide.set_mts(nn, 4)
    wide.close()
    wide = B.Pamd([S.make_peptide(1806, 120)], R_target=16, T0=700.0, dt=0.0005, nu=1.0, seed=1,
                  precision=B.PAMD_FP32)
    with pytest.raises(B.PamdError):
        wide.export_configs(0, 0, 4)
    wide.close()
    nn.close()
