"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every entry point include/pmace.h declares, and rejects bad arguments before
touching a device."""
import ctypes
import os
import re

import pytest

from conftest import ROOT
from paper_2111_14240_amd import pmace as P

HEADER = os.path.join(ROOT, "include", "pmace.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(pmace_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(P.LIB_PATH):
        pytest.fail("libpmace.so is not built (run __graft_entry__.build())")
    return P.load_library()


def test_every_declared_symbol_is_exported(lib):
    names = _declared()
    assert "pmace_init" in names and "pmace_iterate" in names and "pmace_reconstruct" in names
    for n in names:
        assert hasattr(lib, n), n


def test_status_strings(lib):
    for s in range(7):
        assert P.pmace_status_str(s) not in ("", "unknown status")
    assert P.pmace_status_str(99) == "unknown status"


def _fp(**kw):
    base = dict(n1=128, n2=128, np_=32, num_pos=36, alpha=0.5)
    base.update(kw)
    return P.pmace_footprint(P.make_params(**base))


def test_footprint_formula(lib):
    J, np_, n = 36, 32, 128
    fp = _fp()
    # PMACE, Np <= 128: states 8 B + amplitudes 4 B per patch pixel (no staged
    # patches), object images 36 B per pixel (Lambda^-1, accumulator, S, xbar,
    # xhat), probe tables 48 B per probe pixel, positions, tile tables
    lower = J * np_ * np_ * 12 + n * n * 36 + np_ * np_ * 48 + J * 8
    # gather tiles are (16 / k) x w pixels with k in {1, 2, 4} and w in {32, 64}
    # (tuned build parameters)
    tiles = (n // 4) * (n // 32)
    tables = tiles * 24 + J * (31 // 4 + 2) * (31 // 32 + 2) * 4 + J * 8
    nred = n * n // 4096
    assert lower <= fp <= lower + tables + nred * 40 + 1024 + 26 * 256
    # SHARP+ keeps its weighted frames of every position in the stage buffer
    sharp = P.pmace_footprint(P.make_params(128, 128, 32, 36, 0.5, method=1, beta=0.75))
    assert J * np_ * np_ * 8 <= sharp - fp <= J * np_ * np_ * 8 + 256
    # Np = 256 stages one chunk of patches between its passes: at most `chunk`
    # positions, evened out over the chunks (1600 = 25 x 64 = 13 chunks of <= 124)
    a = P.pmace_footprint(P.make_params(1024, 1024, 256, 1600, 0.5, chunk=64))
    b = P.pmace_footprint(P.make_params(1024, 1024, 256, 1600, 0.5, chunk=128))
    stage = (124 - 64) * 256 * 256 * 8
    tile_tables = (25 - 13) * 256 * 32 * 24    # fewer chunks, fewer tile slots (at most)
    row_items = (25 - 13) * 1024 * 16          # and fewer row items of the row-spectrum consensus
    assert stage - tile_tables - row_items - 4096 <= b - a <= stage + 4096


@pytest.mark.parametrize("kw", [dict(np_=0), dict(num_pos=0), dict(n1=16), dict(alpha=-1.0),
                                dict(alpha=float("nan")), dict(rho=0.0), dict(rho=1.0),
                                dict(kappa=-0.5), dict(kappa=float("inf")), dict(flags=0x10),
                                dict(flags=0x2 | 0x8), dict(flags=0x4 | 0x8), dict(flags=0x2 | 0x4),
                                dict(chunk=-1), dict(np_=40)])
def test_invalid_params_rejected(lib, kw):
    assert _fp(**kw) == 0
    st, ctx = P.pmace_init(P.make_params(**{**dict(n1=128, n2=128, np_=32, num_pos=36, alpha=0.5), **kw}),
                           1, 1, 1, None, 1, 1 << 30, None)
    expect = P.PMACE_EUNSUPPORTED if kw == dict(np_=40) else P.PMACE_EINVAL
    assert st == expect and not ctx.value


def test_init_argument_checks_before_device(lib):
    prm = P.make_params(128, 128, 32, 36, 0.5)
    st, _ = P.pmace_init(prm, None, 1, 1, None, 1, 1 << 30, None)
    assert st == P.PMACE_EINVAL
    st, _ = P.pmace_init(prm, 1, 1, 1, None, 1, 16, None)
    assert st == P.PMACE_ENOMEM
    assert P.pmace_iterate(None, 1) == P.PMACE_ESTATE
    assert P.pmace_sync(None) == P.PMACE_ESTATE
    assert P.pmace_fft2(40, 1, 1, 1, 0, None) == P.PMACE_EUNSUPPORTED
    assert P.pmace_fft2(32, -1, 1, 1, 0, None) == P.PMACE_EINVAL
    P.pmace_destroy(None)


def test_batch_argument_checks(lib):
    assert P.pmace_batch_footprint([]) == 0
    st, b = P.pmace_batch_create([], P.pmace_stop_rule(1e-4, 2, 10), 1, 1 << 20)
    assert st == P.PMACE_EINVAL and not b.value
    assert P.pmace_batch_step(None, 1) == P.PMACE_ESTATE
    st, *_ = P.pmace_batch_poll(None, 1)
    assert st == P.PMACE_ESTATE
    assert P.pmace_set_reference(None, None, None) == P.PMACE_ESTATE
    st, _ = P.pmace_nrmse(None)
    assert st == P.PMACE_ESTATE
    st, _ = P.pmace_data_fit(None)
    assert st == P.PMACE_ESTATE
    st, *_ = P.pmace_batch_poll_fit(None, 1)
    assert st == P.PMACE_ESTATE
    P.pmace_batch_destroy(None)


@pytest.mark.parametrize("method,beta", [(2, 0.5), (-1, 0.5), (1, -0.1), (1, 1.5), (1, float("nan"))])
def test_method_parameters_checked(lib, method, beta):
    prm = P.make_params(128, 128, 32, 36, 0.5, method=method, beta=beta)
    assert P.pmace_footprint(prm) == 0
    st, _ = P.pmace_init(prm, 1, 1, 1, None, 1, 1 << 30, None)
    assert st == P.PMACE_EINVAL
    ok = P.make_params(128, 128, 32, 36, 0.5, method=P.PMACE_METHOD_SHARP_PLUS, beta=0.75)
    assert P.pmace_footprint(ok) > 0


def test_binding_shares_pytorch_hip_runtime():
    """Loading the library through the binding in a fresh process, before
    anything else imported PyTorch, maps one HIP runtime: the one PyTorch's
    device pointers belong to."""
    import subprocess
    import sys
    code = ("from paper_2111_14240_amd import pmace; pmace.load_library(); "
            "print(len({l.split()[-1] for l in open('/proc/self/maps') if 'libamdhip64' in l}))")
    out = subprocess.run([sys.executable, "-c", code], cwd=ROOT, capture_output=True, text=True,
                         timeout=300)
    assert out.returncode == 0, out.stderr
    assert out.stdout.strip().splitlines()[-1] == "1"


def test_simulate_static_checks_before_device(lib):
    """The allocation-free simulate entry point rejects bad arguments and
    sizes beyond its static scratch before touching a device."""
    L = lib
    mx = int(L.pmace_simulate_static_max_bytes())
    assert mx == (64 << 20) - 256
    big_j = mx // (256 * 256 * 8) + 1                        # one position too many for Np = 256
    one = ctypes.c_void_p(1)
    assert L.pmace_simulate_static(1024, 1024, 256, big_j, one, one, one, 0.0, 1, one, None,
                                   None) == P.PMACE_ENOMEM
    assert L.pmace_simulate_static(128, 128, 32, 4, None, one, one, 0.0, 1, one, None, None) == P.PMACE_EINVAL
    assert L.pmace_simulate_static(128, 128, 33, 4, one, one, one, 0.0, 1, one, None,
                                   None) == P.PMACE_EUNSUPPORTED
    assert L.pmace_simulate_static(128, 128, 32, 4, one, one, one, float("nan"), 1, one, None,
                                   None) == P.PMACE_EINVAL


def test_patches_per_workgroup_range(lib):
    """pmace_params.ppw: 0 (the build's default) or a power of two within the
    side's maximum (1024 threads per workgroup); anything else is EINVAL, so the
    footprint query returns 0."""
    fp = lambda np_, ppw, n=256: P.pmace_footprint(P.make_params(n, n, np_, 9, 0.5, ppw=ppw))
    for np_, top in ((32, 8), (48, 4), (64, 2), (96, 1), (128, 1), (256, 1)):
        assert fp(np_, 0) > 0
        k = 1
        while k <= top:
            assert fp(np_, k) == fp(np_, 0), (np_, k)
            k *= 2
        assert fp(np_, 2 * top) == 0, (np_, 2 * top)
    assert fp(32, 3) == 0 and fp(32, -1) == 0 and fp(48, 6) == 0
