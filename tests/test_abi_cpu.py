"""CPU checks of the C-ABI library: it loads, exports every declared symbol, validates
configurations and matches the struct layout of include/sacc.h.  No GPU work."""

import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "sacc.h")


@pytest.fixture(scope="module")
def nv():
    import paper_2309_02156_amd.native as native

    if not os.path.exists(native.LIB_PATH):
        from paper_2309_02156_amd import build

        build.build()
    native.lib()
    return native


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(sa_[a-z_]+)\s*\(", text)))


def test_every_declared_symbol_is_exported(nv):
    names = declared_functions()
    assert len(names) >= 9
    out = subprocess.run(["nm", "-D", "--defined-only", nv.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(re.findall(r"\s[TW]\s+(sa_\w+)$", out, flags=re.M))
    assert set(names) <= exported, set(names) - exported
    assert set(nv.EXPORTS) == set(names)


def _cfg(nv, **over):
    kw = dict(n=4096, M=10, s=20, sketch=0, projection=0, solver=0, restart=30, tol=1e-10, maxit=100,
              precision=0, inner_tol=1e-4, max_refine=10, guess=0, rank_tol_sketch=0.0,
              rank_tol_chol=0.0, seed=0, poll=0, inner_maxit=0)
    kw.update(over)
    return nv.SaConfig(**kw)


def test_workspace_sizes_and_validation(nv):
    L = nv.lib()
    b = ctypes.c_size_t(0)
    assert L.sa_workspace_bytes(ctypes.byref(_cfg(nv)), ctypes.byref(b)) == 0
    small = b.value
    # history + basis + CG vectors at least
    assert small >= 8 * (4096 * 10 * 2 + 3 * 4096)
    assert L.sa_workspace_bytes(ctypes.byref(_cfg(nv, solver=1)), ctypes.byref(b)) == 0
    assert b.value > small   # GMRES(30) basis is larger than CG's three vectors
    bad = [dict(M=0), dict(M=33), dict(s=5), dict(s=300), dict(sketch=1, n=1000), dict(sketch=1, n=16, s=20, M=4),
           dict(solver=1, restart=0), dict(solver=1, restart=65), dict(tol=0.0), dict(tol=-1.0),
           dict(maxit=-1), dict(guess=7), dict(n=0), dict(sketch=5), dict(projection=3), dict(projection=2), dict(precision=4),
           dict(precond=2), dict(precond=-1)]
    for over in bad:
        assert L.sa_workspace_bytes(ctypes.byref(_cfg(nv, **over)), ctypes.byref(b)) == nv.SA_EINVAL, over
    assert L.sa_workspace_bytes(None, ctypes.byref(b)) == nv.SA_EINVAL


def test_null_handles_and_status_strings(nv):
    L = nv.lib()
    assert L.sa_destroy_sequence(None) == nv.SA_EINVAL
    assert L.sa_push_solution(None, None, None) == nv.SA_ESTATE
    assert L.sa_initial_guess(None, None, None, None, None, None) == nv.SA_ESTATE
    assert L.sa_solve(None, None, None, None, None, None) == nv.SA_ESTATE
    assert L.sa_step(None, None, None, None, None, None) == nv.SA_ESTATE
    assert L.sa_spmv(None, None, None, None) == nv.SA_EINVAL
    assert L.sa_copy_state(None, 0, None, 0, None) == nv.SA_ESTATE
    nb = ctypes.c_size_t(0)
    assert L.sa_state_bytes(None, ctypes.byref(nb)) == nv.SA_ESTATE
    assert L.sa_export_state(None, None, 0, None) == nv.SA_ESTATE
    assert L.sa_import_state(None, None, 0, None) == nv.SA_ESTATE
    for code in (0, 1, -1, -2, -3, -4, -5, -6):
        s = L.sa_status_string(code).decode()
        assert s and s != "unknown status"
    assert L.sa_status_string(99).decode() == "unknown status"
    # measurement and predictor entry points validate before touching the device
    cnt = ctypes.c_int32(0)
    assert L.sa_profile_enable(None, 1) == nv.SA_ESTATE
    assert L.sa_profile_read(None, None, 0, ctypes.byref(cnt)) == nv.SA_ESTATE
    assert L.sa_learned_attach(None, None, 8) == nv.SA_ESTATE
    assert L.sa_set_time(None, 0.0) == nv.SA_ESTATE
    assert L.sa_mlp_destroy(None) == nv.SA_EINVAL
    assert L.sa_mlp_forward(None, None, 1, None, None) == nv.SA_EINVAL
    assert L.sa_mlp_train_step(None, None, None, 1, None, None) == nv.SA_EINVAL
    assert L.sa_mlp_get(None, 0, None, 0, None) == nv.SA_EINVAL
    assert L.sa_mlp_set_scaling(None, None, None, None, None) == nv.SA_EINVAL
    m = ctypes.c_void_p(0)
    bad = nv.SaMlpConfig(n_in=4, n_hidden=8, n_layers=9, n_out=2, max_batch=4, lr=1e-3, beta1=0.9, beta2=0.999,
                         eps=1e-8, reserved=0)
    w = (ctypes.c_float * 16)()
    assert L.sa_mlp_create(ctypes.byref(bad), w, ctypes.byref(m)) == nv.SA_EINVAL
    bad.n_layers, bad.max_batch = 2, 0
    assert L.sa_mlp_create(ctypes.byref(bad), w, ctypes.byref(m)) == nv.SA_EINVAL
    assert L.sa_mlp_create(None, w, ctypes.byref(m)) == nv.SA_EINVAL
    h = ctypes.c_void_p(0)
    ws = ctypes.create_string_buffer(64)
    # misaligned / undersized workspaces are rejected before any device call
    assert L.sa_init_sequence(ctypes.byref(_cfg(nv)), None, 0, None, ctypes.byref(h)) == nv.SA_EINVAL
    addr = (ctypes.addressof(ws) + 255) // 256 * 256
    assert L.sa_init_sequence(ctypes.byref(_cfg(nv)), ctypes.c_void_p(addr), 16, None,
                              ctypes.byref(h)) == nv.SA_ENOMEM


def test_struct_layout_matches_header(nv, tmp_path):
    src = tmp_path / "layout.c"
    src.write_text(r"""
#include <stdio.h>
#include <stddef.h>
#include "sacc.h"
#define P(T, f) printf(#T "." #f " %zu\n", offsetof(T, f));
int main(void) {
  printf("sa_config %zu\nsa_csr %zu\nsa_info %zu\nsa_kernel_prof %zu\n", sizeof(sa_config), sizeof(sa_csr),
         sizeof(sa_info), sizeof(sa_kernel_prof));
  P(sa_config, tol) P(sa_config, seed) P(sa_config, poll) P(sa_config, rank_tol_chol)
  P(sa_csr, val_dev) P(sa_csr, val_is_fp32) P(sa_info, relres0) P(sa_info, ms_solve)
  P(sa_kernel_prof, launches) P(sa_kernel_prof, ms) P(sa_kernel_prof, bytes)
  P(sa_info, used_learned) P(sa_mlp_config, lr) P(sa_mlp_config, eps) P(sa_mlp_config, max_batch)
  printf("sa_mlp_config %zu\n", sizeof(sa_mlp_config));
  return 0;
}
""")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    lines = dict(l.split() for l in subprocess.run([str(exe)], capture_output=True, text=True).stdout.splitlines())
    assert int(lines["sa_config"]) == ctypes.sizeof(nv.SaConfig)
    assert int(lines["sa_csr"]) == ctypes.sizeof(nv.SaCsr)
    assert int(lines["sa_info"]) == ctypes.sizeof(nv.SaInfo)
    assert int(lines["sa_kernel_prof"]) == ctypes.sizeof(nv.SaKernelProf)
    assert int(lines["sa_mlp_config"]) == ctypes.sizeof(nv.SaMlpConfig)
    for key, v in lines.items():
        if "." in key:
            struct, field = key.split(".")
            cls = {"sa_config": nv.SaConfig, "sa_csr": nv.SaCsr, "sa_info": nv.SaInfo,
                   "sa_kernel_prof": nv.SaKernelProf, "sa_mlp_config": nv.SaMlpConfig}[struct]
            assert getattr(cls, field).offset == int(v), key


def test_product_path_does_not_touch_the_oracle():
    """The HIP binding never imports the oracle, and the oracle never imports the binding."""
    pkg = os.path.join(ROOT, "paper_2309_02156_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".cpp", ".hip", ".h")):
                text = open(os.path.join(dirpath, f)).read()
                assert not re.search(r"^\s*(from|import)\s+oracle", text, flags=re.M), f
                assert "oracle/" not in text, f
    for f in os.listdir(os.path.join(ROOT, "oracle")):
        if f.endswith(".py"):
            text = open(os.path.join(ROOT, "oracle", f)).read()
            assert "paper_2309_02156_amd" not in text, f


def test_static_solve_limits(nv):
    """The allocation-free solve reports its fixed scratch, rejects configurations that do
    not fit it (SA_ETOOBIG) or that it does not serve (SA_EINVAL) before any device work."""
    L = nv.lib()
    need, cap = ctypes.c_size_t(0), ctypes.c_size_t(0)
    assert L.sa_static_scratch_bytes(ctypes.byref(_cfg(nv, n=4096)), ctypes.byref(need), ctypes.byref(cap)) == 0
    assert cap.value == 32 << 20 and 4 * 8 * 4096 < need.value < cap.value
    big = _cfg(nv, n=1 << 21)
    assert L.sa_static_scratch_bytes(ctypes.byref(big), ctypes.byref(need), ctypes.byref(cap)) == 0
    assert need.value > cap.value
    info = nv.SaInfo()
    dummy = ctypes.c_void_p(256)
    csr = nv.SaCsr(1 << 21, 7 << 21, dummy, dummy, dummy, 0, 0)
    assert L.sa_solve_static(ctypes.byref(big), ctypes.byref(csr), dummy, dummy, ctypes.byref(info),
                             None) == nv.SA_ETOOBIG
    gm = _cfg(nv, n=1 << 17, solver=1, restart=30)   # 32 vectors of 2^17 doubles: 32 MiB
    assert L.sa_static_scratch_bytes(ctypes.byref(gm), ctypes.byref(need), ctypes.byref(cap)) == 0
    assert need.value > cap.value
    mixed = _cfg(nv, n=4096, precision=1)
    csr = nv.SaCsr(4096, 7 * 4096, dummy, dummy, dummy, 1, 0)
    assert L.sa_solve_static(ctypes.byref(mixed), ctypes.byref(csr), dummy, dummy, ctypes.byref(info),
                             None) == nv.SA_EINVAL
    assert L.sa_solve_static(ctypes.byref(_cfg(nv, n=4096)), ctypes.byref(csr), None, dummy, ctypes.byref(info),
                             None) == nv.SA_EINVAL
    assert b"fixed scratch" in L.sa_status_string(nv.SA_ETOOBIG)
