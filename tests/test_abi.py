"""The C-ABI library builds, loads and exports every declared symbol; host-side
argument validation rejects bad inputs before any device work (no GPU)."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def L():
    from paper_2405_14492_amd import fsa
    if not os.path.exists(fsa.LIB_PATH):
        from paper_2405_14492_amd import build
        build.build(verbose=False)
    return fsa.load_library()


def declared_symbols():
    src = open(os.path.join(ROOT, "include", "fsa.h")).read()
    return sorted(set(re.findall(r"^\s*(?:fsa_status|void|int64_t|double|const char\*)\s*(fsa_\w+)\s*\(", src, re.M)))


def test_every_declared_symbol_is_exported(L):
    names = declared_symbols()
    assert len(names) >= 12
    for nm in names:
        assert hasattr(L, nm), nm
    from paper_2405_14492_amd import fsa
    assert set(fsa.EXPORTED) == set(names)


def test_header_constants_match_binding(L):
    from paper_2405_14492_amd import fsa
    src = open(os.path.join(ROOT, "include", "fsa.h")).read()
    for nm, val in (("FSA_FP64", fsa.FP64), ("FSA_MIXED_FP32", fsa.MIXED_FP32),
                    ("FSA_MIXED_BF16A", fsa.MIXED_BF16A), ("FSA_CV_NONE", fsa.CV_NONE), ("FSA_CV_ONE", fsa.CV_ONE),
                    ("FSA_CV_OPT", fsa.CV_OPT), ("FSA_CV_OPT_PRINTED", fsa.CV_OPT_PRINTED)):
        assert re.search(r"\b%s = %d\b" % (nm, val), src), nm
    assert int(re.search(r"#define FSA_PROFILE_ALL (0x[0-9a-f]+)", src).group(1), 16) == fsa.PROFILE_ALL
    assert fsa.make_options(profile=True).profile == fsa.PROFILE_ALL
    assert fsa.make_options(profile=1).profile == 1
    assert fsa.make_options().profile == 0
    assert fsa.make_options().control_variate == 0 and fsa.make_options(control_variate=2).control_variate == 2
    # the options struct keeps its size: control_variate fills the hole after num_probes
    assert fsa.fsa_options.control_variate.offset == 4 and fsa.fsa_options.seed.offset == 8


def test_struct_layouts(L):
    from paper_2405_14492_amd import fsa
    # fsa_options: 2 x int32, uint64, double, 6 x int32, double, void*, 2 x int32
    assert ctypes.sizeof(fsa.fsa_options) == 72
    assert ctypes.sizeof(fsa.fsa_theta) == 32
    o = fsa.fsa_options()
    L.fsa_default_options(ctypes.byref(o))
    assert o.num_probes == 50 and o.cg_rel_tol == 1e-8 and o.max_iter == 1000 and o.precision == 0
    assert o.graph == 0
    assert o.control_variate == 0
    assert o.fp32_products == fsa.F32P_SPLIT


@pytest.mark.parametrize("case", ["n1", "d3", "m0", "m_gt_n", "gamma0", "sigma2_0", "rho_neg", "cov_bad", "probes0",
                                  "cv_bad", "f32p_bad"])
def test_invalid_arguments_rejected_on_host(L, case):
    from paper_2405_14492_amd import fsa
    n, d, m, gamma = 10, 2, 3, 0.1
    theta = [0, 1.0, 0.1, 0.1]
    opt = fsa.make_options()
    if case == "n1":
        n = 1
        m = 1
    elif case == "d3":
        d = 3
    elif case == "m0":
        m = 0
    elif case == "m_gt_n":
        m = 11
    elif case == "gamma0":
        gamma = 0.0
    elif case == "sigma2_0":
        theta[3] = 0.0
    elif case == "rho_neg":
        theta[2] = -1.0
    elif case == "cov_bad":
        theta[0] = 7
    elif case == "probes0":
        opt.num_probes = 0
    elif case == "cv_bad":
        opt.control_variate = 4
    elif case == "f32p_bad":
        opt.fp32_products = 2
    locs = np.zeros((max(n, 1), d))
    y = np.zeros(max(n, 1))
    ind = np.zeros((max(m, 1), d))
    th = fsa.make_theta(theta)
    ctx = ctypes.c_void_p()
    s = L.fsa_build(locs.ctypes.data, n, d, y.ctypes.data, ctypes.byref(th), ind.ctypes.data, m, gamma,
                    ctypes.byref(opt), ctypes.byref(ctx))
    assert s == 1
    assert not ctx.value
    assert len(L.fsa_last_error()) > 0


@pytest.mark.parametrize("case", ["n0", "m0", "m513", "mv33", "mv_neg", "kind_bad", "rho0", "s1_neg", "null_w"])
def test_vecchia_invalid_arguments_rejected_on_host(L, case):
    """fsa_vecchia_build_dev checks sizes and parameters before it touches
    any pointer or the device (the buffers here are host memory, never read)."""
    n, m, kind, s1, rho, mv = 10, 3, 1, 1.0, 0.1, 5
    if case == "n0":
        n = 0
    elif case == "m0":
        m = 0
    elif case == "m513":
        m = 513
    elif case == "mv33":
        mv = 33
    elif case == "mv_neg":
        mv = -1
    elif case == "kind_bad":
        kind = 9
    elif case == "rho0":
        rho = 0.0
    elif case == "s1_neg":
        s1 = -1.0
    buf = np.zeros(2 * 1024)
    w = None if case == "null_w" else buf.ctypes.data
    h = ctypes.c_void_p()
    s = L.fsa_vecchia_build_dev(buf.ctypes.data, n, buf.ctypes.data, m, kind, s1, rho, mv, w, None, ctypes.byref(h))
    assert s == 1
    assert not h.value
    assert len(L.fsa_last_error()) > 0


def test_vecchia_null_handle(L):
    buf = np.zeros(16)
    d = ctypes.c_double()
    assert L.fsa_vecchia_apply_dev(None, 0, buf.ctypes.data, 1, 1, buf.ctypes.data, 1) == 1
    assert L.fsa_vecchia_solve_logdet_dev(None, buf.ctypes.data, buf.ctypes.data, 4, 0, 1e-6, 10, 0,
                                          ctypes.byref(d), None) == 1
    assert L.fsa_vecchia_factor_dev(None, None, None, None) == 1
    assert L.fsa_vecchia_destroy(None) == 0


def test_set_allocator_validates_on_host(L):
    """Both callbacks or neither; neither restores the library's own pool.
    No device memory is touched."""
    from paper_2405_14492_amd import fsa
    alloc = fsa.ALLOC_FN(lambda nbytes, stream, user: None)
    assert L.fsa_set_allocator(alloc, fsa.RELEASE_FN(), None) == 1
    assert len(L.fsa_last_error()) > 0
    assert L.fsa_set_allocator(fsa.ALLOC_FN(), fsa.RELEASE_FN(), None) == 0


def test_nll_grad_dev_rejects_null_handle(L):
    assert L.fsa_nll_grad_dev(None, None, None, None, None) == 1
