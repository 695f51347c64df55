"""CPU checks of the C ABI boundary: the library loads and exports every entry
point declared in include/pamd.h, the binding's structures match the header's
field lists, and the build does not leave packed-FP32 instructions behind."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pamd.h")
LIB = os.path.join(ROOT, "paper_1806_06016_amd", "libpamd.so")


def _declared_functions():
    txt = open(HEADER).read()
    return sorted(set(re.findall(r"\b(pamd_[a-z0-9_]+)\s*\(", txt)))


def _struct_fields(name):
    txt = open(HEADER).read()
    m = re.search(r"typedef struct " + name + r" \{(.*?)\} " + name + ";", txt, re.S)
    body = re.sub(r"/\*.*?\*/", "", m.group(1), flags=re.S)
    fields = []
    for decl in body.split(";"):
        decl = decl.strip()
        if not decl:
            continue
        decl = re.sub(r"\bconst\b", "", decl)
        parts = decl.split(None, 1)
        for nm in parts[1].split(","):
            fields.append(nm.strip().lstrip("*").strip())
    return fields


@pytest.mark.skipif(not os.path.exists(LIB), reason="libpamd.so not built")
def test_library_exports_every_declared_entry_point():
    lib = ctypes.CDLL(LIB)
    names = _declared_functions()
    assert "pamd_init" in names and "pamd_md_steps" in names and "pamd_resample" in names
    assert "pamd_observables" in names
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_structs_match_header():
    from paper_1806_06016_amd import pamd as B
    for cname, py in [("pamd_system", B.pamd_system), ("pamd_params", B.pamd_params),
                      ("pamd_obs", B.pamd_obs), ("pamd_run_scalars", B.pamd_run_scalars),
                      ("pamd_family_stats", B.pamd_family_stats)]:
        assert [f for f, _ in py._fields_] == _struct_fields(cname), cname


def test_binding_exports_list_matches_header():
    from paper_1806_06016_amd import pamd as B
    assert sorted(B.EXPORTS) == _declared_functions()


@pytest.mark.skipif(not os.path.exists(LIB), reason="libpamd.so not built")
def test_query_sizes_is_host_only_and_validates():
    """pamd_query_sizes needs no GPU; it rejects bad descriptors."""
    import numpy as np
    from paper_1806_06016_amd import pamd as B
    from pamd_inputs import systems as S
    lib = B.load_library()
    keep = []
    sysd = S.c2_system()
    s = B.make_system_struct(sysd, keep)
    p = B.pamd_params()
    p.R_target, p.R_cap, p.T0, p.dt, p.nu, p.seed, p.precision = 1000, 1100, 700.0, 0.001, 1.0, 1, 1
    sb, wb = ctypes.c_size_t(), ctypes.c_size_t()
    assert lib.pamd_query_sizes(ctypes.byref(s), 1, ctypes.byref(p), ctypes.byref(sb), ctypes.byref(wb)) == 0
    # 2 ping-pong slabs of R_cap x 6 x 80 floats dominate the state
    assert sb.value >= 2 * 1100 * 6 * 80 * 4
    p.R_cap = 10
    assert lib.pamd_query_sizes(ctypes.byref(s), 1, ctypes.byref(p), ctypes.byref(sb),
                                ctypes.byref(wb)) == B.PAMD_ERR_ARG
    p.R_cap = 1100
    for mode, want in [(B.PAMD_RESAMPLE_MULTINOMIAL, 0), (B.PAMD_RESAMPLE_NONE, 0), (3, B.PAMD_ERR_ARG),
                       (-1, B.PAMD_ERR_ARG)]:
        p.resampling = mode
        assert lib.pamd_query_sizes(ctypes.byref(s), 1, ctypes.byref(p), ctypes.byref(sb),
                                    ctypes.byref(wb)) == want
    p.resampling = B.PAMD_RESAMPLE_NEAREST
    p.thermostat = 2                           # no such bath
    assert lib.pamd_query_sizes(ctypes.byref(s), 1, ctypes.byref(p), ctypes.byref(sb),
                                ctypes.byref(wb)) == B.PAMD_ERR_ARG
    p.thermostat = B.PAMD_THERMOSTAT_LANGEVIN
    assert lib.pamd_query_sizes(ctypes.byref(s), 1, ctypes.byref(p), ctypes.byref(sb),
                                ctypes.byref(wb)) == 0
    two_s = (B.pamd_system * 2)(s, s)
    two_p = (B.pamd_params * 2)(p, p)
    two_p[1].thermostat = B.PAMD_THERMOSTAT_ANDERSEN   # one bath per context
    assert lib.pamd_query_sizes(two_s, 2, two_p, ctypes.byref(sb), ctypes.byref(wb)) == B.PAMD_ERR_ARG
    p.thermostat = B.PAMD_THERMOSTAT_ANDERSEN
    bad = S.c2_system()
    bad.dih_delta = bad.dih_delta + 0.3        # only 0 / pi phases are supported
    sb2 = B.make_system_struct(bad, keep)
    assert lib.pamd_query_sizes(ctypes.byref(sb2), 1, ctypes.byref(p), ctypes.byref(sb),
                                ctypes.byref(wb)) == B.PAMD_ERR_ARG
    big = S.make_peptide(1806, 120)            # above the register tiles: wide layout, 128-atom slabs
    s3 = B.make_system_struct(big, keep)
    assert lib.pamd_query_sizes(ctypes.byref(s3), 1, ctypes.byref(p), ctypes.byref(sb),
                                ctypes.byref(wb)) == 0
    assert sb.value >= 2 * 1100 * 6 * 128 * 4
    p.precision = 0                            # FP64 is limited to 32 atoms
    assert lib.pamd_query_sizes(ctypes.byref(s3), 1, ctypes.byref(p), ctypes.byref(sb),
                                ctypes.byref(wb)) == B.PAMD_ERR_ARG
    p.precision = 1
    s4 = B.make_system_struct(S.make_peptide(7, 300), keep)
    s4.n_atoms = B.MAX_ATOMS + 1               # beyond the wide layout
    assert lib.pamd_query_sizes(ctypes.byref(s4), 1, ctypes.byref(p), ctypes.byref(sb),
                                ctypes.byref(wb)) == B.PAMD_ERR_ARG
    # the wide kernels' LJ class table holds 25 distinct (sigma, epsilon) pairs;
    # the register-tile layout (per-pair tables) takes any number
    for n, k, want in [(120, B.WIDE_LJ_CLASSES, 0), (120, B.WIDE_LJ_CLASSES + 1, B.PAMD_ERR_ARG), (75, 26, 0), (75, 75, 0)]:
        m = S.make_peptide(1806, n)
        m.sigma = 0.3 * (1.0 + 1e-3 * (np.arange(n) % k))
        m.epsilon = np.full(n, 0.5)
        sm = B.make_system_struct(m, keep)
        assert lib.pamd_query_sizes(ctypes.byref(sm), 1, ctypes.byref(p), ctypes.byref(sb),
                                    ctypes.byref(wb)) == want, (n, k)


def test_binding_fails_loudly_without_library(tmp_path):
    from paper_1806_06016_amd import pamd as B
    saved = B._lib
    B._lib = None
    try:
        with pytest.raises(RuntimeError, match="missing"):
            B.load_library(str(tmp_path / "nope.so"))
    finally:
        B._lib = saved


def test_surrogate_parameter_count_matches_layout():
    """PAMD_NN_PARAMS = |W1| + |b1| + |W2| + |b2| + |w3| + |b3| for the
    256 -> 128 -> 128 -> 1 network, in the header and the binding."""
    import numpy as np
    txt = open(os.path.join(ROOT, "include", "pamd.h")).read()
    vals = {k: int(v) for k, v in re.findall(r"#define (PAMD_NN_\w+) (\d+)", txt)}
    F, H = vals["PAMD_NN_FEATURES"], vals["PAMD_NN_HIDDEN"]
    assert vals["PAMD_NN_PARAMS"] == F * H + H + H * H + H + H + 1
    from paper_1806_06016_amd import pamd as B
    assert B.NN_PARAMS == vals["PAMD_NN_PARAMS"] and B.NN_FEATURES == F and B.NN_HIDDEN == H
    assert B.NN_STATIC_ROWS == vals["PAMD_NN_STATIC_ROWS"]
    w = {"W1": np.zeros((F, H)), "b1": np.zeros(H), "W2": np.zeros((H, H)), "b2": np.zeros(H),
         "w3": np.arange(H, dtype=float), "b3": np.ones(1)}
    back = B.unpack_params(B.pack_params(w))
    assert all(np.array_equal(back[k], w[k]) for k in w)
