"""C-ABI checks that need no GPU: the library loads, exports every function
the public header declares, its structs match the Python mirrors, and its
host-side argument validation rejects bad calls before touching a device."""
import ctypes
import os
import subprocess

import pytest

from paper_2309_04623_amd import build as libbuild
from paper_2309_04623_amd import nmf

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

EXPECTED = {
    "nmf_create", "nmf_destroy", "nmf_status_string", "nmf_last_error", "nmf_params_default",
    "nmf_workspace_bytes", "nmf_init_uniform", "nmf_objective", "nmf_build_basis", "nmf_project",
    "nmf_project_ragged", "nmf_subtract", "nmf_profile_enable", "nmf_profile_get",
    "nmf_device_clock_khz", "nmf_warmstart_param_count", "nmf_warmstart_init",
    "nmf_warmstart_pool", "nmf_warmstart_step", "nmf_warmstart_train", "nmf_warmstart_infer",
    "nmf_autotune_report", "nmf_closest_frames", "nmf_best_factor", "nmf_build_basis_sequential",
    "nmf_warm_fallbacks", "nmf_frame_iters", "nmf_frame_visits",
}


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(nmf.LIB_PATH):
        libbuild.build()
    return nmf.lib()


def test_header_declares_the_boundary():
    assert EXPECTED <= set(nmf.header_functions())


def test_every_declared_function_is_exported(L):
    raw = ctypes.CDLL(nmf.LIB_PATH)
    for name in nmf.header_functions():
        assert hasattr(raw, name), name


def test_struct_layout_matches_c(tmp_path):
    """Compile a probe against the header with the host C compiler and compare
    sizes/offsets with the ctypes mirrors."""
    src = tmp_path / "probe.c"
    src.write_text(
        '#include <stdio.h>\n#include <stddef.h>\n#include "nmf_mi355x.h"\n'
        "int main(void){printf(\"%zu %zu %zu %zu %zu %zu %zu\\n\", sizeof(nmf_params), "
        "offsetof(nmf_params, tol), offsetof(nmf_params, seed), offsetof(nmf_params, floor_eps), "
        "sizeof(nmf_report), offsetof(nmf_report, objective), offsetof(nmf_report, elapsed_ms));"
        "return 0;}\n")
    exe = tmp_path / "probe"
    subprocess.run(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)],
                   check=True)
    vals = [int(x) for x in subprocess.run([str(exe)], capture_output=True, text=True,
                                           check=True).stdout.split()]
    P, R = nmf.Params, nmf.Report
    assert vals == [ctypes.sizeof(P), P.tol.offset, P.seed.offset, P.floor_eps.offset,
                    ctypes.sizeof(R), R.objective.offset, R.elapsed_ms.offset]


def test_status_strings(L):
    for code in (0, -1, -2, -3, -4, -5, -6, -7, -8, 1, 2):
        assert L.nmf_status_string(code)
    assert L.nmf_status_string(12345) == b"unknown status"


def test_params_default(L):
    p = nmf.Params()
    L.nmf_params_default(ctypes.byref(p))
    assert p.struct_size == ctypes.sizeof(nmf.Params)
    assert p.k == 1 and p.precision == 0 and p.max_iter == 200
    assert abs(p.floor_eps - 1e-30) < 1e-36


FAKE = 0x10000  # never dereferenced: validation fails first


def _prm(L, **kw):
    p = nmf.Params()
    L.nmf_params_default(ctypes.byref(p))
    for k, v in kw.items():
        setattr(p, k, v)
    return p


def _bb(L, n=64, p=128, prm=None, V=FAKE, M=FAKE + 8, W_out=FAKE + 16, H_out=FAKE + 24, h=None,
        rep=None):
    prm = prm or _prm(L, k=4)
    return L.nmf_build_basis(h, V, M, n, p, ctypes.byref(prm), None, None, W_out, H_out, None,
                             rep, None)


def test_build_basis_validation(L):
    assert _bb(L, V=None) == nmf.NMF_ERR_ARG
    assert _bb(L, n=0) == nmf.NMF_ERR_SHAPE
    assert _bb(L, p=-3) == nmf.NMF_ERR_SHAPE
    assert _bb(L, prm=_prm(L, k=0)) == nmf.NMF_ERR_ARG
    assert _bb(L, prm=_prm(L, k=65)) == nmf.NMF_ERR_ARG  # k > min(n, p)
    assert _bb(L, prm=_prm(L, k=4, struct_size=12)) == nmf.NMF_ERR_ARG
    assert b"struct_size" in L.nmf_last_error()
    assert _bb(L, prm=_prm(L, k=4, precision=7)) == nmf.NMF_ERR_ARG
    assert _bb(L, prm=_prm(L, k=4, max_iter=-1)) == nmf.NMF_ERR_ARG
    assert _bb(L, prm=_prm(L, k=4, tol=-1.0)) == nmf.NMF_ERR_ARG
    assert _bb(L, prm=_prm(L, k=4, floor_eps=float("nan"))) == nmf.NMF_ERR_ARG
    assert _bb(L, W_out=FAKE) == nmf.NMF_ERR_ARG  # W_out aliases V
    assert b"aliasing" in L.nmf_last_error()
    assert _bb(L, W_out=FAKE + 16, H_out=FAKE + 16) == nmf.NMF_ERR_ARG
    bad = nmf.Report()
    bad.struct_size = 3
    assert _bb(L, rep=ctypes.byref(bad)) == nmf.NMF_ERR_ARG
    # everything valid but the handle
    assert _bb(L) == nmf.NMF_ERR_ARG
    assert b"handle" in L.nmf_last_error()


def test_project_and_subtract_validation(L):
    prm = _prm(L, k=4)
    P = ctypes.byref(prm)
    assert L.nmf_project(None, FAKE, 4, 100, None, FAKE, 3, P, None, FAKE + 8, None, None,
                         None) == nmf.NMF_ERR_ARG
    assert L.nmf_project(None, FAKE, 5, 100, FAKE + 4, FAKE + 8, 3, P, None, FAKE + 12, None, None,
                         None) == nmf.NMF_ERR_ARG  # params.k != k
    assert L.nmf_project(None, FAKE, 4, 100, FAKE + 4, FAKE + 8, 0, P, None, FAKE + 12, None, None,
                         None) == nmf.NMF_ERR_SHAPE
    assert L.nmf_project(None, FAKE, 4, 100, FAKE + 4, FAKE + 8, 3, P, None, FAKE + 4, None, None,
                         None) == nmf.NMF_ERR_ARG  # C_out aliases T
    # the per-frame stop rule exists for the masked-Gram form only
    tp = _prm(L, k=4)
    tp.tol, tp.check_every = 1e-4, 10
    assert L.nmf_project(None, FAKE, 4, 100, FAKE + 4, FAKE + 8, 3, ctypes.byref(tp), None,
                         FAKE + 12, None, None, None) == nmf.NMF_ERR_UNSUPPORTED
    assert L.nmf_frame_iters(None, None, 0) == nmf.NMF_ERR_ARG
    assert L.nmf_frame_visits(None, None, 0) == nmf.NMF_ERR_ARG
    assert L.nmf_subtract(None, FAKE, FAKE + 4, FAKE + 8, FAKE + 12, 2, 4, 100, None, None, None,
                          None) == nmf.NMF_ERR_ARG
    assert L.nmf_subtract(None, FAKE, FAKE + 4, FAKE + 8, FAKE + 12, 2, 0, 100, None, None,
                          FAKE + 16, None) == nmf.NMF_ERR_ARG
    assert L.nmf_subtract(None, FAKE, FAKE + 4, FAKE + 8, FAKE + 12, 2, 4, 100, None, None,
                          FAKE + 8, None) == nmf.NMF_ERR_ARG  # resid aliases T
    assert L.nmf_subtract(None, FAKE, FAKE + 4, FAKE + 8, FAKE + 12, 2, 4, 100, None, None,
                          FAKE + 16, None) == nmf.NMF_ERR_ARG  # handle


def test_init_and_objective_validation(L):
    assert L.nmf_init_uniform(None, 1, 0, 0, 5, FAKE, None) == nmf.NMF_ERR_SHAPE
    assert L.nmf_init_uniform(None, 1, -1, 3, 5, FAKE, None) == nmf.NMF_ERR_ARG
    assert L.nmf_init_uniform(None, 1, 0, 3, 5, None, None) == nmf.NMF_ERR_ARG
    out = ctypes.c_double()
    assert L.nmf_objective(None, FAKE, FAKE, FAKE, FAKE, 10, 20, 11, 0, ctypes.addressof(out),
                           None) == nmf.NMF_ERR_ARG
    assert L.nmf_objective(None, FAKE, FAKE, FAKE, FAKE, 10, 20, 3, 5, ctypes.addressof(out),
                           None) == nmf.NMF_ERR_ARG


def test_create_without_device_fails_cleanly(L):
    try:
        import torch
        if torch.cuda.is_available():
            pytest.skip("a GPU is present")
    except ImportError:
        pass
    h = ctypes.c_void_p()
    rc = L.nmf_create(0, ctypes.byref(h))
    assert rc in (nmf.NMF_ERR_HIP, nmf.NMF_ERR_ARG)
    assert not h.value
    assert L.nmf_destroy(None) == 0


def test_project_ragged_validation(L):
    prm = _prm(L, k=4)
    P = ctypes.byref(prm)

    def call(h=None, H=FAKE, k=4, p=100, f=3, off=FAKE + 4, nnz=10, pix=FAKE + 8, val=FAKE + 12,
             wt=None, prm_=P, C=FAKE + 16):
        return L.nmf_project_ragged(h, H, k, p, f, off, nnz, pix, val, wt, prm_, None, C, None,
                                    None, None)
    assert call(off=None) == nmf.NMF_ERR_ARG
    assert call(pix=None) == nmf.NMF_ERR_ARG
    assert call(nnz=-1) == nmf.NMF_ERR_SHAPE
    assert call(f=0) == nmf.NMF_ERR_SHAPE
    assert call(k=5) == nmf.NMF_ERR_ARG           # params.k != k
    big = _prm(L, k=201)
    assert call(k=201, p=1000, prm_=ctypes.byref(big)) == nmf.NMF_ERR_UNSUPPORTED
    assert call(C=FAKE + 12) == nmf.NMF_ERR_ARG    # C_out aliases val
    assert call() == nmf.NMF_ERR_ARG               # handle
    assert b"handle" in L.nmf_last_error()


def test_warmstart_layout_and_validation(L):
    assert L.nmf_warmstart_param_count(100) == 1024 * 512 + 512 + 512 * 512 + 512 + 512 * 100 + 100
    assert L.nmf_warmstart_param_count(0) == 0
    assert L.nmf_warmstart_init(None, None, 4, 0, None) == nmf.NMF_ERR_ARG
    assert L.nmf_warmstart_init(None, FAKE, 0, 0, None) == nmf.NMF_ERR_ARG
    assert L.nmf_warmstart_step(None, FAKE, FAKE, FAKE, FAKE, FAKE, 0, 4, 0, 0.0, 1, None, None,
                                None) == nmf.NMF_ERR_SHAPE
    assert L.nmf_warmstart_step(None, FAKE, FAKE, FAKE, FAKE, FAKE, 8, 4, 0, 1e-3, 0, None, None,
                                None) == nmf.NMF_ERR_ARG
    assert L.nmf_warmstart_train(None, FAKE, FAKE, FAKE, FAKE, FAKE, 100, 4, 0, 1, 8, 0.0, 0, None,
                                 None) == nmf.NMF_ERR_ARG
    assert L.nmf_warmstart_pool(None, FAKE, FAKE, 2, 0, 5, FAKE, FAKE, None) == nmf.NMF_ERR_SHAPE


def test_pipeline_calls_validation(L):
    """Reference selection, best factor and the sequential build reject bad
    arguments on the host, before any device work."""
    F = FAKE
    # closest frames: n_sel out of range, null index output, handle
    assert L.nmf_closest_frames(None, F, F + 4, 10, 100, F + 8, F + 12, 2, 0, None, F + 16,
                                None) == nmf.NMF_ERR_ARG
    assert L.nmf_closest_frames(None, F, F + 4, 10, 100, F + 8, F + 12, 2, 11, None, F + 16,
                                None) == nmf.NMF_ERR_ARG
    assert L.nmf_closest_frames(None, F, F + 4, 10, 100, F + 8, F + 12, 2, 3, None, None,
                                None) == nmf.NMF_ERR_ARG
    assert L.nmf_closest_frames(None, F, F + 4, 0, 100, F + 8, F + 12, 2, 3, None, F + 16,
                                None) == nmf.NMF_ERR_SHAPE
    assert L.nmf_closest_frames(None, F, F + 4, 10, 100, F + 8, F + 12, 2, 3, None, F + 16,
                                None) == nmf.NMF_ERR_ARG
    assert b"handle" in L.nmf_last_error()
    # best factor: empty range, k out of range
    assert L.nmf_best_factor(None, F, F + 4, F + 8, F + 12, None, 2, 3, 100, 2.0, 1.0, F + 16,
                             None) == nmf.NMF_ERR_ARG
    assert L.nmf_best_factor(None, F, F + 4, F + 8, F + 12, None, 2, 0, 100, 0.0, 1.0, F + 16,
                             None) == nmf.NMF_ERR_ARG
    assert L.nmf_best_factor(None, F, F + 4, F + 8, F + 12, None, 2, 3, 100, 0.0, 1.0, None,
                             None) == nmf.NMF_ERR_ARG
    # sequential build: k above the supported width, k > min(n, p)
    prm = _prm(L, k=225)
    assert L.nmf_build_basis_sequential(None, F, F + 4, 300, 1000, ctypes.byref(prm), F + 8,
                                        F + 12, None, None, None) == nmf.NMF_ERR_UNSUPPORTED
    prm = _prm(L, k=40)
    assert L.nmf_build_basis_sequential(None, F, F + 4, 30, 1000, ctypes.byref(prm), F + 8,
                                        F + 12, None, None, None) == nmf.NMF_ERR_ARG
    prm = _prm(L, k=4)
    assert L.nmf_build_basis_sequential(None, F, F + 4, 30, 1000, ctypes.byref(prm), F + 8,
                                        F + 12, None, None, None) == nmf.NMF_ERR_ARG
    assert b"handle" in L.nmf_last_error()
