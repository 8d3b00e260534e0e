"""CPU checks of the C ABI: the library loads, exports every declared symbol,
and the host-side validation / workspace sizing behave as documented (no
device work is done here)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pcop.h")


def _declared_functions():
    text = open(HEADER).read()
    names = set(re.findall(r"^(?:pcop_status|void|const char\*)\s+(pcop_[a-z0-9_]+)\s*\(", text, re.M))
    return sorted(names)


@pytest.fixture(scope="module")
def lib():
    from paper_2410_22686_amd import pcop
    if not os.path.exists(pcop.LIB_PATH):
        from paper_2410_22686_amd import build
        build.build()
    return pcop.load_library()


def test_every_declared_symbol_is_exported(lib):
    names = _declared_functions()
    assert len(names) >= 14
    for n in names:
        assert hasattr(lib, n), n
    from paper_2410_22686_amd import pcop
    assert sorted(pcop.EXPORTED) == names


def _prob(dim=2, nx=31, nt=32, gammas=(1e-4,), eps=-1.0, coeff=None):
    from paper_2410_22686_amd import pcop
    p = pcop.c_problem()
    p.dim, p.nx, p.nt, p.T, p.batch = dim, nx, nt, 1.0, len(gammas)
    arr = (ctypes.c_double * len(gammas))(*gammas)
    p.gamma = ctypes.cast(arr, ctypes.POINTER(ctypes.c_double))
    p.eps = eps
    if coeff is None:
        p.coeff_kind, p.coeff = pcop.PCOP_COEFF_ONE, None
    else:
        p.coeff_kind = pcop.PCOP_COEFF_HALFGRID
        p.coeff = coeff.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    p._keep = arr
    return p


def _opts(lib, **kw):
    from paper_2410_22686_amd import pcop
    o = pcop.c_options()
    lib.pcop_default_options(ctypes.byref(o))
    for k, v in kw.items():
        setattr(o, k, v)
    return o


def test_defaults_validate(lib):
    from paper_2410_22686_amd import pcop
    o = _opts(lib)
    assert (o.precision, o.spatial, o.side, o.restart, o.maxit) == (0, 0, 0, 30, 300)
    assert o.rtol == 1e-8
    assert lib.pcop_validate(ctypes.byref(_prob()), ctypes.byref(o)) == pcop.PCOP_OK


@pytest.mark.parametrize("field,value,status", [
    ("dim", 4, 1), ("nx", 0, 1), ("nt", 1, 1), ("T", 0.0, 1), ("eps", 1.5, 1),
    ("nx", 30, 2),  # sine transforms need nx + 1 = 2^k
])
def test_invalid_problems_are_rejected(lib, field, value, status):
    p = _prob()
    setattr(p, field, value)
    assert lib.pcop_validate(ctypes.byref(p), ctypes.byref(_opts(lib))) == status
    assert len(lib.pcop_last_error()) > 0


def test_invalid_options_are_rejected(lib):
    p = _prob()
    for kw in [dict(restart=0), dict(restart=41), dict(maxit=0), dict(rtol=0.0), dict(side=7),
               dict(precision=1, side=0), dict(graph=1, graph_chunk=0), dict(time_cols=2),
               dict(time_cols=-2), dict(time_cols=128), dict(time_cols=-128), dict(dst_kernel=6), dict(dst_kernel=-1), dict(tune=2),
               dict(precond=2), dict(precond=-1), dict(kkt_jchunk=65), dict(kkt_jchunk=-65),
               dict(krylov_blocks=4097), dict(krylov_blocks=-2), dict(gs_update=3),
               dict(mg_smoother=3), dict(mg_smoother=-1)]:
        assert lib.pcop_validate(ctypes.byref(p), ctypes.byref(_opts(lib, **kw))) == 1, kw


def test_kernel_choice_options_validate(lib):
    p = _prob()
    o = _opts(lib)
    assert (o.time_cols, o.dst_kernel, o.tune) == (0, 0, 0)
    for kw in [dict(time_cols=-1), dict(time_cols=4), dict(time_cols=8), dict(time_cols=16),
               dict(time_cols=-4), dict(time_cols=-8), dict(time_cols=-16), dict(time_cols=32), dict(time_cols=-32), dict(time_cols=64), dict(time_cols=-64), dict(precond=1),
               dict(kkt_jchunk=4), dict(kkt_jchunk=-16), dict(krylov_blocks=512), dict(gs_update=2),
               dict(dst_kernel=1), dict(dst_kernel=2), dict(dst_kernel=3), dict(dst_kernel=4), dict(dst_kernel=5), dict(tune=1),
               dict(mg_smoother=1), dict(mg_smoother=2)]:
        assert lib.pcop_validate(ctypes.byref(p), ctypes.byref(_opts(lib, **kw))) == 0, kw


def test_every_time_length_up_to_2048_validates(lib):
    """Every n = nt - 1 in 1..2048 has a time-pass kernel in both precisions:
    radix plans whose tiles fit LDS, otherwise the chirp-z transform (M up to
    4096), which also takes long smooth lengths such as n = 1152 or 2048.
    Beyond that the chirp-z length exceeds 4096 and setup refuses."""
    from paper_2410_22686_amd import pcop
    for precision, side in ((pcop.PCOP_FP64, pcop.PCOP_RIGHT), (pcop.PCOP_MIXED, pcop.PCOP_FLEXIBLE)):
        o = _opts(lib, precision=precision, side=side)
        bad = [n for n in range(1, 2049)
               if lib.pcop_validate(ctypes.byref(_prob(nx=3, nt=n + 1)), ctypes.byref(o)) != pcop.PCOP_OK]
        assert bad == [], (precision, bad[:10])
        for n in (2049, 2050, 4096):
            assert lib.pcop_validate(ctypes.byref(_prob(nx=3, nt=n + 1)), ctypes.byref(o)) == 2, (precision, n)


def test_finite_element_mass_rules(lib):
    """PCOP_MASS_Q1 (Section 1 with M_m != I) runs with a = 1, sine
    transforms and the epsilon-circulant preconditioner; other combinations
    are refused before any launch, and unknown values are invalid."""
    from paper_2410_22686_amd import pcop
    p = _prob(dim=2, nx=7, nt=8)
    p.mass = pcop.PCOP_MASS_Q1
    assert lib.pcop_validate(ctypes.byref(p), ctypes.byref(_opts(lib))) == 0
    assert lib.pcop_validate(ctypes.byref(p), ctypes.byref(_opts(lib, precision=1, side=2))) == 0
    assert lib.pcop_validate(ctypes.byref(p), ctypes.byref(_opts(lib, spatial=1, side=2))) == 2
    assert lib.pcop_validate(ctypes.byref(p), ctypes.byref(_opts(lib, precond=1))) == 2
    p.mass = 2
    assert lib.pcop_validate(ctypes.byref(p), ctypes.byref(_opts(lib))) == 1


def test_gamma_must_be_positive(lib):
    assert lib.pcop_validate(ctypes.byref(_prob(gammas=(1e-4, -1.0))), ctypes.byref(_opts(lib))) == 1
    assert lib.pcop_validate(ctypes.byref(_prob(gammas=(float("nan"),))), ctypes.byref(_opts(lib))) == 1


def test_variable_coefficient_rules(lib):
    import numpy as np
    nx = 7
    a = np.ones((2 * nx + 1) ** 3)
    p = _prob(dim=3, nx=nx, nt=8, coeff=a)
    assert lib.pcop_validate(ctypes.byref(p), ctypes.byref(_opts(lib))) == 1          # DST needs a = 1
    assert lib.pcop_validate(ctypes.byref(p), ctypes.byref(_opts(lib, spatial=1))) == 0
    a[5] = 0.0
    assert lib.pcop_validate(ctypes.byref(p), ctypes.byref(_opts(lib, spatial=1))) == 1
    p2 = _prob(dim=3, nx=6, nt=8, coeff=np.ones(13 ** 3))
    assert lib.pcop_validate(ctypes.byref(p2), ctypes.byref(_opts(lib, spatial=1))) == 1  # not 2^p - 1


def test_workspace_size_scales_with_problem(lib):
    sizes = []
    for nx, nt in [(31, 32), (63, 64)]:
        nb = ctypes.c_size_t()
        assert lib.pcop_workspace_size(ctypes.byref(_prob(nx=nx, nt=nt)), ctypes.byref(_opts(lib)),
                                       ctypes.byref(nb)) == 0
        sizes.append(nb.value)
        vec = 8 * 2 * nx * nx * (nt - 1)
        # 31 basis slots + 2 temporaries + the spectrum
        assert nb.value >= 33 * vec
    assert sizes[1] > 7 * sizes[0]
    nbf = ctypes.c_size_t()
    assert lib.pcop_workspace_size(ctypes.byref(_prob()), ctypes.byref(_opts(lib, side=2)), ctypes.byref(nbf)) == 0
    assert nbf.value > sizes[0]  # flexible GMRES keeps Z as well


def test_status_strings(lib):
    for s in range(6):
        assert len(lib.pcop_status_string(s)) > 0


def test_ideal_preconditioner_has_no_time_transform_limit(lib):
    """P of eq. matrix_P needs no FFT along time, so long horizons validate."""
    p = _prob(nx=31, nt=4096)
    assert lib.pcop_validate(ctypes.byref(p), ctypes.byref(_opts(lib))) == 2
    assert lib.pcop_validate(ctypes.byref(p), ctypes.byref(_opts(lib, precond=1))) == 0
