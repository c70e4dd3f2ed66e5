"""Host-side checks of the C ABI (no GPU needed, no compute calls)."""

import ctypes
import os
import re
import subprocess

import pytest

import paper_2511_15196_amd as P
from paper_2511_15196_amd import _abi

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "phi4pmc.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[a-z_0-9]+\s*\*?\s+([a-z_0-9]+)\s*\(", text, flags=re.M)
    return sorted(set(names))


def test_header_declares_the_boundary():
    names = declared_functions()
    for n in ["smc_init", "smc_mutate", "smc_reweight_resample", "ns_step", "logz"]:
        assert n in names


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(_abi.library_path)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_covers_every_symbol():
    assert set(declared_functions()) == set(_abi.SIGNATURES)


def _c_layout(struct, fields):
    src = "#include <stdio.h>\n#include <stddef.h>\n#include \"phi4pmc.h\"\nint main(void){\n"
    src += f'printf("%zu\\n", sizeof({struct}));\n'
    for f in fields:
        src += f'printf("%zu\\n", offsetof({struct}, {f}));\n'
    src += "return 0;}\n"
    return src


@pytest.mark.parametrize("struct,cls", [("phi4_smc_config", _abi.SmcConfig),
                                        ("phi4_ns_config", _abi.NsConfig)])
def test_ctypes_layout_matches_c(tmp_path, struct, cls):
    fields = [f for f, _ in cls._fields_]
    cfields = ["lambda" if f == "lambda_" else f for f in fields]
    c = tmp_path / "layout.c"
    c.write_text(_c_layout(struct, cfields))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(c), "-o", str(exe)], check=True)
    out = [int(x) for x in subprocess.run([str(exe)], capture_output=True, text=True,
                                          check=True).stdout.split()]
    assert out[0] == ctypes.sizeof(cls)
    for f, off in zip(fields, out[1:]):
        assert getattr(cls, f).offset == off, f


def test_workspace_sizes_and_validation():
    good = P.SmcConfig(L=8, N=4096, m2=-4.0, lambda_=8.0, ess_frac=0.5, n_steps=20,
                       acc_target=0.3, eps0=0.0, seed=0, run=0, precision=0)
    assert P.smc_workspace_bytes(good) > 4096 * 64 * 4
    for bad in [dict(L=65), dict(N=1), dict(ess_frac=0.0), dict(ess_frac=1.5), dict(precision=7),
                dict(n_steps=-1), dict(kernel=3), dict(kernel=1, precision=1),
                dict(kernel=1, L=33), dict(kernel=2, precision=1), dict(kernel=2, n_leapfrog=-1),
                dict(kernel=2, n_leapfrog=1001)]:
        cfg = P.SmcConfig(**{**{f: getattr(good, f) for f, _ in good._fields_}, **bad})
        assert P.smc_workspace_bytes(cfg) == 0
    # the independence sampler adds its own scratch (mean, whitening factor, residuals)
    ind = P.SmcConfig(**{**{f: getattr(good, f) for f, _ in good._fields_}, "kernel": 1})
    assert P.smc_workspace_bytes(ind) > P.smc_workspace_bytes(good) + 64 * 64 * 4
    ind.L = 32
    assert P.smc_workspace_bytes(ind) > 0
    hmc = P.SmcConfig(**{**{f: getattr(good, f) for f, _ in good._fields_}, "kernel": 2})
    assert P.smc_workspace_bytes(hmc) > P.smc_workspace_bytes(good)   # site variances
    hmc.L, hmc.n_leapfrog = 64, 1000
    assert P.smc_workspace_bytes(hmc) > 0
    ns = P.NsConfig(L=8, n_live=4096, k_delete=2048, n_steps=40, m2=-4.0, lambda_=8.0,
                    prior_var=4.0, term_frac=1e-3, acc_target=0.3, eps0=0.0, seed=0, run=0,
                    precision=1)
    assert P.ns_workspace_bytes(ns) > 0
    ns.k_delete = 4095
    assert P.ns_workspace_bytes(ns) == 0
    assert P.phi4_step_workspace_bytes(4096, 64) > 0
    assert P.phi4_step_workspace_bytes(16, 4097) == 0
    # the large-lattice sweep needs scratch for normals, proposals and counts
    assert P.phi4_step_workspace_bytes(64, 1024) > 64 * 1024 * 8


def test_invalid_calls_fail_before_touching_the_gpu():
    lib = P.lib()
    h = ctypes.c_void_p()
    bad = P.SmcConfig(L=0, N=10)
    rc = lib.smc_init(ctypes.byref(bad), None, None, None, 0, None, ctypes.byref(h))
    assert rc == P.PHI4_EINVAL and b"L" in lib.phi4_last_error()
    assert lib.smc_mutate(None, None) == P.PHI4_EINVAL
    assert lib.ns_step(None, None) == P.PHI4_EINVAL
    assert lib.phi4_action(None, 5, 0, 0.0, 0.0, None, None, None) == P.PHI4_EINVAL
    assert lib.phi4_destroy(None) == P.PHI4_OK
