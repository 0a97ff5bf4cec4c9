"""The C ABI library loads and exports every entry point of include/nmodes.h;
host-only entry points (filter design) behave, and errors are reported."""
import ctypes as C
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "nmodes.h")).read()
    return sorted(set(re.findall(r"\b(nm_[a-z_]+)\s*\(", src)) - {"nm_status"})


@pytest.fixture(scope="module")
def lib():
    import paper_1906_11082_amd as nm
    return nm.load_library()


def test_exports_every_declared_symbol(lib):
    names = _declared()
    assert len(names) >= 15
    for n in names:
        assert hasattr(lib, n), n


def test_binding_covers_header():
    import paper_1906_11082_amd as nm
    assert sorted(nm.EXPORTED) == _declared()


def test_filter_coeffs_match_oracle(lib):
    import paper_1906_11082_amd as nm
    from oracle import solve as S
    for (a, b, lo, hi, m) in [(0.5, 40, 0, 3700, 40), (1, 60, -0.3, 3e5, 333), (10, 20, 0, 50, 0)]:
        mu = nm.filter_coeffs(a, b, lo, hi, m)
        ref, _, _ = S.filter_coeffs(a, b, lo, hi, m)
        assert np.abs(mu - ref).max() < 1e-14


def test_filter_degree_rule_properties(lib):
    """The chosen degree keeps the filter below 1 % of its window-edge level
    beyond the guard point (checked with the oracle's polynomial); modes 1
    (damping below a) and 2 (null factor)."""
    import paper_1906_11082_amd as nm
    from oracle import solve as S
    for a, b, lo, hi, nul in [(1, 60, 0, 3e4, True), (0.5, 40, 0, 3700, False)]:
        m = nm.filter_degree(a, b, lo, hi, 0.5, 2 if nul else 1)
        mu, c, e = S.filter_coeffs(a, b, lo, hi, m)
        f = lambda lam: S.cheb_series(mu, (np.asarray(lam) - c) / e) * (np.asarray(lam) / b if nul else 1)
        lev = min(f(a), f(b))
        lam = np.linspace(1.5 * b, hi, 20000)
        assert np.abs(f(lam)).max() <= 0.01 * lev * (1 + 1e-9)
        mu2, _, _ = S.filter_coeffs(a, b, lo, hi, int(m / 1.15) - 1)
        f2 = lambda lam: S.cheb_series(mu2, (np.asarray(lam) - c) / e) * (np.asarray(lam) / b if nul else 1)
        # a clearly lower degree fails the rule somewhere
        lam2 = np.linspace(1.5 * b, hi, 200000)
        lev2 = min(f2(a), f2(b))
        bad = np.abs(f2(lam2)).max() > 0.01 * lev2
        if not nul:
            lam3 = np.linspace(lo, a - 0.5 * (a - lo), 20000)
            bad = bad or np.abs(f2(lam3)).max() > 0.01 * lev2
        assert bad


def test_errors_are_reported(lib):
    import paper_1906_11082_amd as nm
    with pytest.raises(nm.NMError) as ei:
        nm.filter_coeffs(2.0, 1.0, 0, 10, 5)
    assert ei.value.status == -1 and "invalid" in str(ei.value)
    r = lib.nm_filtered_eig(None, 0.0, 1.0, 1, 1e-8, None, None)
    assert r == -1


def test_filter_degree_upper_only_is_cheaper(lib):
    import paper_1906_11082_amd as nm
    m0 = nm.filter_degree(1, 60, 0, 3e4, 0.5, 0)
    m1 = nm.filter_degree(1, 60, 0, 3e4, 0.5, 1)
    assert m0 < m1


def test_struct_layouts_match_header(tmp_path):
    """The ctypes mirrors of the header's structs have the C compiler's field
    offsets and sizes (a field added to one side only shifts every later one)."""
    import shutil
    import subprocess
    import paper_1906_11082_amd as nm
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    rename = {"_EigResult": {"lam": "lambda"}}
    structs = [(nm._Mesh, "nm_mesh"), (nm._Material, "nm_material"), (nm._Info, "nm_pencil_info"),
               (nm._ApplyOpts, "nm_apply_opts"), (nm._EigOpts, "nm_eig_opts"), (nm._EigResult, "nm_eig_result"),
               (nm._RotResult, "nm_rot_result"), (nm._Request, "nm_request"),
               (nm._ServerResult, "nm_server_result")]
    lines = ['#include <stddef.h>', '#include <stdio.h>', '#include "nmodes.h"', "int main(void) {"]
    want = []
    for cls, cname in structs:
        lines.append('printf("%%zu\\n", sizeof(%s));' % cname)
        want.append(("sizeof", cname, C.sizeof(cls)))
        for f in cls._fields_:
            name = rename.get(cls.__name__, {}).get(f[0], f[0])
            lines.append('printf("%%zu\\n", offsetof(%s, %s));' % (cname, name))
            want.append((cname, name, getattr(cls, f[0]).offset))
    lines += ["return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run([cc, "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = [int(x) for x in subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split()]
    assert len(got) == len(want)
    for (a, b, w), g in zip(want, got):
        assert g == w, (a, b, w, g)


def test_set_allocator_arguments(lib):
    """nm_set_allocator takes both functions or neither (no device call is made)."""
    import paper_1906_11082_amd as nm
    a = nm._ALLOC_FN(lambda n, s, c: None)
    assert lib.nm_set_allocator(a, nm._FREE_FN(), None) == -1
    assert "both" in lib.nm_last_error().decode()
    with pytest.raises(ValueError):
        nm.set_allocator(alloc=lambda n: 0)
    nm.set_allocator(None, None)
    assert lib.nm_last_error().decode() == ""


def test_block_width_guard(lib):
    """Vector blocks are indexed with 32-bit offsets: the widest accepted block
    for n displacement rows keeps n * ncols below 2^32 (the C5-sized body with
    16 windows of 64 columns would not fit), and the query rejects n <= 0."""
    import paper_1906_11082_amd as nm
    for n in (2187, 1_633_791, 5_000_000, 15_000_000):
        k = nm.max_block_columns(n)
        assert k >= 1 and n * k < 2 ** 32 and n * (k + 1) >= 2 ** 32 - 1
    assert nm.max_block_columns(5_000_000) < 16 * 64
    with pytest.raises(nm.NMError) as e:
        nm.max_block_columns(0)
    assert e.value.status == -1


def test_dos_count_and_slices_match_oracle(lib):
    """Host-side density-of-states counts and equal-count slice ends equal the
    oracle's for the same traces (the oracle pins them against exact counts)."""
    import paper_1906_11082_amd as nm
    from oracle import dos as D
    lam = np.sort(np.random.default_rng(5).uniform(0.0, 3.0e3, 900) ** 1.5 / 50.0)
    lmin, lmax = -0.5, 1.01 * lam.max()
    tau = D.exact_traces(lam, lmin, lmax, 700)
    for a, b in [(1.0, 60.0), (5.0, 400.0)]:
        assert abs(nm.dos_count(tau, lmin, lmax, a, b) - D.window_count(tau, lmin, lmax, a, b)) <= 1e-9 * len(lam)
        e1 = nm.dos_slices(tau, lmin, lmax, a, b, 4)
        e2 = D.slice_edges(tau, lmin, lmax, a, b, 4)
        assert np.abs(e1 - e2).max() <= 1e-9 * b
    # weighted traces (null-free): the library's panel quadrature of the 1/lambda
    # series against the oracle's adaptive quadrature
    lam = np.concatenate([np.zeros(3000), lam])
    tw = D.exact_traces(lam, lmin, lmax, 700, weighted=True)
    for a, b in [(1.0, 60.0), (5.0, 400.0)]:
        cw = nm.dos_count(tw, lmin, lmax, a, b, weighted=True)
        assert abs(cw - D.window_count(tw, lmin, lmax, a, b, weighted=True)) <= 1e-8 * len(lam)
        e1 = nm.dos_slices(tw, lmin, lmax, a, b, 3, weighted=True)
        e2 = D.slice_edges(tw, lmin, lmax, a, b, 3, weighted=True)
        assert np.abs(e1 - e2).max() <= 1e-7 * b
    with pytest.raises(nm.NMError):
        nm.dos_count(tw, lmin, lmax, 0.0, 10.0, weighted=True)


def test_block_products_reject_bad_arguments(lib):
    """The dense block products check their sizes on the host before any
    launch: leading dimensions below the used widths, negative sizes, null
    matrices of a non-empty product and an output that is the input."""
    import ctypes as C
    dummy = C.c_void_p(256)  # never dereferenced: every call below fails its checks first
    assert lib.nm_gemm_tn(10, 8, 4, dummy, 7, dummy, 4, dummy, None) == -1       # lda < K
    assert lib.nm_gemm_tn(10, 8, 4, dummy, 8, dummy, 3, dummy, None) == -1       # ldb < q
    assert lib.nm_gemm_tn(-1, 8, 4, dummy, 8, dummy, 4, dummy, None) == -1       # n < 0
    assert lib.nm_gemm_tn(10, 8, 4, None, 8, dummy, 4, dummy, None) == -1        # null A
    assert lib.nm_gemm_nn(10, 8, 4, 1.0, dummy, 8, dummy, 7, 0.0, dummy, 4, None) == -1  # ldc < K
    assert lib.nm_gemm_nn(10, 8, 4, 1.0, dummy, 8, dummy, 8, 0.0, dummy, 3, None) == -1  # ldd < q
    assert lib.nm_gemm_nn(10, 8, 4, 1.0, dummy, 8, dummy, 8, 0.0, None, 4, None) == -1   # null D
    assert lib.nm_gemm_nn(10, 8, 4, 1.0, dummy, 8, C.c_void_p(512), 8, 0.0, dummy, 4, None) == -1  # A == D
    assert "gemm" in lib.nm_last_error().decode() or "null" in lib.nm_last_error().decode()


def test_block_product_wrappers_check_their_tensors():
    """The Python wrappers of the block products accept only 2-D float64
    device tensors with contiguous rows and matching row counts (checked
    before any library call, so this runs without a GPU)."""
    import torch
    import paper_1906_11082_amd as nm
    with pytest.raises(ValueError):
        nm.gemm_tn(torch.zeros((4, 3), dtype=torch.float64), torch.zeros((4, 2), dtype=torch.float64))
    with pytest.raises(ValueError):
        nm.gemm_nn(torch.zeros((4, 3), dtype=torch.float32), torch.zeros((3, 2)))
