"""The C ABI library loads and exports every symbol that include/nep.h declares
(no compute call: this runs without a GPU)."""
import ctypes as C
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "nep.h")


def _declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(nep_[a-z_]+)\s*\(", txt)))


def _lib():
    import paper_2305_08140_amd as nep
    if not os.path.exists(nep.LIB_PATH):
        pytest.skip("libnep_hip.so not built")
    return nep, nep.lib()


def test_header_declares_the_entry_points():
    d = _declared()
    for name in ("nep_create", "nep_destroy", "nep_build_neighbors", "nep_compute_efv", "nep_step_verlet",
                 "nep_status", "nep_strerror"):
        assert name in d


def test_library_exports_every_declared_symbol():
    nep, L = _lib()
    for name in _declared():
        assert hasattr(L, name), name
    assert set(_declared()) == set(nep.EXPORTED)


def test_argument_errors_without_device():
    nep, L = _lib()
    import nep_synth
    m = nep_synth.random_model()
    ptr = C.c_void_p()
    hp = nep.hparams_from(m)
    cfg = nep.Config(1000, 1, 48, 96, 0, 1.0)
    assert L.nep_create(None, C.byref(cfg), C.byref(ptr)) == nep.NEP_E_ARG
    assert L.nep_create(C.byref(hp), C.byref(cfg), None) == nep.NEP_E_ARG
    bad = nep.hparams_from(m)
    bad.n_hidden = 100
    assert L.nep_create(C.byref(bad), C.byref(cfg), C.byref(ptr)) == nep.NEP_E_UNSUPPORTED
    cfg2 = nep.Config(1000, 1, 300, 96, 0, 1.0)   # list capacity above 255
    assert L.nep_create(C.byref(hp), C.byref(cfg2), C.byref(ptr)) == nep.NEP_E_ARG
    assert not ptr.value
    assert L.nep_compute_efv(None, None, None, None) == nep.NEP_E_ARG
    assert L.nep_step_verlet(None, None, None, 1, None, None, None) == nep.NEP_E_ARG
    assert L.nep_population_reserve(None, 4) == nep.NEP_E_ARG
    assert L.nep_population_efv(None, None, 4, None, None, None, None, None, None, None) == nep.NEP_E_ARG
    assert L.nep_snes_sample(0, 10, None, None, None, None, None) == nep.NEP_E_ARG
    assert L.nep_snes_update(1, 10, None, 1, None, None, None, 0.0, 0.0, None) == nep.NEP_E_ARG
    assert L.nep_snes_update(2000, 10, None, 1, None, None, None, 0.0, 0.0, None) == nep.NEP_E_ARG
    L.nep_destroy(None)


def test_strerror_covers_codes():
    nep, L = _lib()
    for code in range(0, -10, -1):
        s = nep.strerror(code)
        assert s and s != "unknown error"
    assert nep.strerror(-99) == "unknown error"


def test_struct_layouts_match_the_header(tmp_path):
    # sizeof and every field offset of the header's structs, compiled with the
    # host C compiler, against the ctypes mirrors of the binding
    import shutil
    import subprocess
    import paper_2305_08140_amd as nep
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    pairs = {"nep_hparams": nep.Hparams, "nep_weights": nep.Weights, "nep_config": nep.Config,
             "nep_system": nep.System, "nep_efv": nep.Efv, "nep_md": nep.Md, "nep_md_stats": nep.MdStats,
             "nep_bcc_ref": nep.BccRef, "nep_defects": nep.Defects, "nep_targets": nep.Targets}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "nep.h"', "int main(void) {"]
    for cname, py in pairs.items():
        lines.append(f'printf("{cname} sizeof %zu\\n", sizeof({cname}));')
        for f in py._fields_:
            lines.append(f'printf("{cname} {f[0]} %zu\\n", offsetof({cname}, {f[0]}));')
    lines.append("return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run([cc, "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = {}
    for ln in subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.splitlines():
        a, b, v = ln.split()
        got[(a, b)] = int(v)
    for cname, py in pairs.items():
        assert got[(cname, "sizeof")] == C.sizeof(py), cname
        for f in py._fields_:
            assert got[(cname, f[0])] == getattr(py, f[0]).offset, (cname, f[0])


def test_split_theta_follows_the_model_layout():
    # the flat parameter vector is split by the context's model sizes: the
    # default model (1057 values) and the paper-size one (16/11 functions on
    # 16/11 Chebyshev terms, 60 descriptors, 100 neurons)
    import torch
    from paper_2305_08140_amd.autograd import split_theta
    import nep_synth
    for m in (nep_synth.random_model(), nep_synth.random_model(size="paper")):
        dim = m.n_rad + m.n_ang * m.l_max
        sizes = (m.n_rad * m.k_rad, m.n_ang * m.k_ang, m.n_hidden * dim, m.n_hidden, m.n_hidden, 1)
        theta = torch.tensor(m.param_vector())
        parts = split_theta(theta, sizes)
        for got, want in zip(parts, (m.c_rad, m.c_ang, m.w0, m.b0, m.w1)):
            assert np.array_equal(got.numpy(), np.asarray(want, dtype=theta.numpy().dtype).ravel())
        assert float(parts[5]) == float(np.asarray(m.b1, dtype=theta.numpy().dtype))
        with pytest.raises(ValueError):
            split_theta(theta[:-1], sizes)
