"""The oracle's C part under AddressSanitizer and UndefinedBehaviorSanitizer
(CPU only): a sanitized build of oracle.c, loaded through the oracle's own
Python wrapper in a child process with the ASan runtime preloaded, runs every
entry point on small cases (forces of every term type and size edge, Andersen
and Langevin MD with collisions, velocities, resampling in all modes, the
adaptive step, a short anneal).  Any sanitizer report fails the test."""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

SCRIPT = r"""
import numpy as np
from oracle import oracle as O
from pamd_inputs import systems as S
for sysd in (S.bead_chain(1), S.bead_chain(2), S.c1_system(), S.branched_pair(), S.gaussian_chain(10),
             S.make_peptide(1806, 33)):
    o = O.OracleSystem(sysd)
    R = 3
    x = np.ascontiguousarray(sysd.x_init[None] + np.random.default_rng(1).normal(0, 0.01, (R,) + sysd.x_init.shape))
    E, F, terms = O.energy_forces(o, x, want_terms=True)
    T = 1.3 if sysd.units == "reduced" else 700.0
    v = O.init_velocities(o, R, T, seed=3, slots=np.array([5, 0, 7]))
    for th in ("andersen", "langevin"):
        xx, vv = x.copy(), v.copy()
        O.md_steps(o, xx, vv, 20, T, 0.001, 5.0, 7, step0=3, slots=np.array([5, 0, 7]), want_collisions=True,
                   thermostat=th)
E = np.random.default_rng(2).normal(0, 3, 1000)
m, S_, S2, lq = O.lse(E, 0.3)
u = O.resample_uniforms(1000, 1, seed=5)
c, tau = O.copy_counts(E, 0.3, 1000, u)
O.multinomial_counts(E, 0.3, O.multinomial_uniforms(700, 1, seed=5))
O.weight_variance(E, 0.3)
O.adaptive_dbeta(E, 2.0, 0.1)
O.anneal(S.c1_system(), 64, 2.0, S.geometric_schedule(2.0, 1.0, 3), theta=20, theta_eq=20, dt=0.002, nu=1.0, seed=1)
O.anneal(S.c1_system(), 64, 2.0, None, theta=20, theta_eq=20, dt=0.002, nu=1.0, seed=1, T_final=1.0,
         resampling="multinomial")
print("sanitized oracle ok")
"""


def test_oracle_c_is_clean_under_asan_and_ubsan(tmp_path):
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("gcc not available")
    asan = subprocess.run([gcc, "-print-file-name=libasan.so"], capture_output=True, text=True).stdout.strip()
    if not os.path.isabs(asan) or not os.path.exists(asan):
        pytest.skip("ASan runtime not available")
    lib = str(tmp_path / "liboracle_san.so")
    flags = ["-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
             "-fno-sanitize-recover=undefined", "-fopenmp", "-fPIC", "-shared"]
    subprocess.check_call([gcc, *flags, "-o", lib, os.path.join(ROOT, "oracle", "oracle.c"), "-lm"])
    env = dict(os.environ, PAMD_ORACLE_LIB=lib, LD_PRELOAD=asan, OMP_NUM_THREADS="2",
               ASAN_OPTIONS="detect_leaks=0", UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1",
               PYTHONPATH=ROOT)
    r = subprocess.run([sys.executable, "-c", SCRIPT], cwd=ROOT, env=env, capture_output=True, text=True,
                       timeout=600)
    report = r.stderr[-4000:]
    assert r.returncode == 0, report
    assert "AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr, report
    assert "sanitized oracle ok" in r.stdout
