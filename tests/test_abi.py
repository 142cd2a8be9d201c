"""CPU tests of the C ABI: the library loads, exports every function the
header declares, and rejects bad arguments before touching a device."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_2204_08988_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "dpmm.h")


def _declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(dpmm_[a-z_]+)\s*\(", txt)))


def test_header_and_binding_agree():
    assert _declared() == sorted(_lib.EXPORTS)


def test_library_exports_every_declared_symbol():
    L = _lib.lib()
    for name in _declared():
        assert hasattr(L, name), name


def _cfg(**kw):
    d = kw.pop("d", 2)
    m = np.zeros(d)
    psi = np.eye(d) if d <= 1024 else None  # a Gaussian prior is not read past d = 128
    cfg = _lib.Config()
    cfg.family = kw.pop("family", _lib.GAUSSIAN)
    cfg.d = d
    cfg.k_max = kw.pop("k_max", 16)
    cfg.burn_out = kw.pop("burn_out", 0)
    cfg.alpha = kw.pop("alpha", 1.0)
    cfg.kappa = kw.pop("kappa", 1.0)
    cfg.nu = kw.pop("nu", d + 3.0)
    psi = kw.pop("psi", psi)
    keep = [m, psi]
    cfg.m = m.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    cfg.psi = psi.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) if psi is not None else None
    beta = kw.pop("beta", None)
    if beta is not None:
        keep.append(beta)
        cfg.beta = beta.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    for name in ("gamma_shape", "gamma_rate"):
        arr = kw.pop(name, None)
        if arr is not None:
            keep.append(arr)
            setattr(cfg, name, arr.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    cfg.seed = 1
    cfg.precision = kw.pop("precision", _lib.FP32)
    cfg.merge_form = kw.pop("merge_form", _lib.MERGE_PAPER)
    cfg.learned = kw.pop("learned", 0)
    cfg.sparse = kw.pop("sparse", 0)
    assert not kw
    return cfg, keep


@pytest.mark.parametrize("kw,status", [
    (dict(family=7), -1),
    (dict(d=0), -1),
    (dict(d=129), -1),
    (dict(k_max=0), -1),
    (dict(k_max=5000), -1),
    (dict(burn_out=-1), -1),
    (dict(alpha=0.0), -1),
    (dict(alpha=float("nan")), -1),
    (dict(kappa=-1.0), -1),
    (dict(nu=0.5), -1),
    (dict(precision=9), -1),
    (dict(precision=1, d=2), -1),
    (dict(precision=2, d=48), -1),
    (dict(merge_form=3), -1),
    (dict(learned=-1), -1),
    (dict(learned=3, d=2), -1),
    (dict(learned=33, d=64), -1),
    (dict(learned=1, family=_lib.MULTINOMIAL, d=4, beta=np.ones(4)), -1),
    (dict(psi=np.array([[1.0, 2.0], [2.0, 1.0]])), -4),
    (dict(psi=np.array([[1.0, 0.5], [0.4, 1.0]])), -4),
    (dict(family=_lib.MULTINOMIAL, d=4), -1),
    (dict(family=_lib.MULTINOMIAL, d=3, beta=np.array([1.0, 0.0, 1.0])), -1),
    (dict(family=_lib.POISSON, d=3), -1),
    (dict(family=_lib.POISSON, d=3, gamma_shape=np.ones(3)), -1),
    (dict(family=_lib.POISSON, d=2, gamma_shape=np.array([1.0, 0.0]), gamma_rate=np.ones(2)), -1),
    (dict(family=_lib.POISSON, d=2, gamma_shape=np.ones(2), gamma_rate=np.array([1.0, float("inf")])), -1),
    (dict(family=_lib.POISSON, d=129, gamma_shape=np.ones(129), gamma_rate=np.ones(129)), -1),
    (dict(learned=1, family=_lib.POISSON, d=4, gamma_shape=np.ones(4), gamma_rate=np.ones(4)), -1),
    (dict(sparse=2, family=_lib.MULTINOMIAL, d=4, beta=np.ones(4)), -1),
    (dict(sparse=1), -1),  # Gaussian
    (dict(sparse=1, family=_lib.MULTINOMIAL, d=2 ** 20 + 1, beta=np.ones(2 ** 20 + 1)), -1),
    (dict(sparse=1, family=_lib.POISSON, d=2 ** 20 + 1, gamma_shape=np.ones(2 ** 20 + 1),
          gamma_rate=np.ones(2 ** 20 + 1)), -1),
    (dict(sparse=1, family=_lib.MULTINOMIAL, d=300, beta=np.ones(300), precision=1), -1),
    (dict(family=_lib.MULTINOMIAL, d=300, beta=np.ones(300)), -1),  # dense rows: V <= 128
])
def test_create_rejects_bad_config_before_device(kw, status):
    L = _lib.lib()
    cfg, keep = _cfg(**kw)
    ctx = ctypes.c_void_p()
    s = L.dpmm_create(ctypes.byref(cfg), None, ctypes.byref(ctx))
    assert s == status, L.dpmm_last_error(None)
    assert not ctx.value
    assert len(L.dpmm_last_error(None)) > 0


def test_null_arguments():
    L = _lib.lib()
    ctx = ctypes.c_void_p()
    assert L.dpmm_create(None, None, ctypes.byref(ctx)) == -1
    cfg, keep = _cfg()
    assert L.dpmm_create(ctypes.byref(cfg), None, None) == -1
    assert L.dpmm_sample_params(None, 1) == -1
    assert L.dpmm_step(None, None, 0, 1, None, None, None) == -1
    L.dpmm_destroy(None)
    assert L.dpmm_status_string(-3) == b"capacity exceeded"
    assert L.dpmm_mlp_n_params(None) == 0
    assert L.dpmm_mlp_set_weights(None, None) == -1
    assert L.dpmm_mlp_forward(None, None, 0, None) == -1
    assert L.dpmm_mlp_grad(None, None, None, 0, None, None) == -1
    assert L.dpmm_learned_move(None, None, 0, 1, None, None, None, None) == -1
    assert L.dpmm_mlp_train(None, None, 0, None, None, 1, 1, 1e-3, None) == -1
    assert L.dpmm_set_features(None, None, 0, None, 0, -1, None, None, 0, None) == -1


def test_struct_layouts_match_header(tmp_path):
    """Every field offset and the size of the three ABI structs, as a C
    compiler lays them out from include/dpmm.h, equal the ctypes binding's."""
    import shutil
    import subprocess
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    structs = {"dpmm_config": _lib.Config, "dpmm_iter_info": _lib.IterInfo, "dpmm_learned_info": _lib.LearnedInfo,
               "dpmm_fit_options": _lib.FitOptions, "dpmm_csr": _lib.CSR}
    lines = ["#include <stddef.h>", "#include <stdio.h>", '#include "dpmm.h"', "int main(void) {"]
    for cname, py in structs.items():
        lines.append(f'  printf("{cname} size %zu\\n", sizeof({cname}));')
        for f, _ in py._fields_:
            lines.append(f'  printf("{cname} {f} %zu\\n", offsetof({cname}, {f}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run([cc, "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {tuple(l.split()[:2]): int(l.split()[2]) for l in out if l}
    for cname, py in structs.items():
        assert got[(cname, "size")] == ctypes.sizeof(py), cname
        for f, _ in py._fields_:
            assert got[(cname, f)] == getattr(py, f).offset, (cname, f)
