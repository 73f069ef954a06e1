"""Host-side checks of the C ABI: no GPU needed, no compute calls.

The library must load, export every function include/corr2d.h declares, and
reject invalid arguments before any device work.
"""
import ctypes
import os
import re
import subprocess

import numpy as np
import pytest

from paper_1808_00685_amd import binding as B

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "corr2d.h")

pytestmark = pytest.mark.skipif(not os.path.exists(B.LIB_PATH),
                                reason="libcorr2d.so not built (run __graft_entry__.build())")


def declared_functions():
    """Functions the library exports: every corr2d_* declared in the header
    except the static inline layout helpers, which live in the header."""
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    inline = set(re.findall(r"static inline \w+ (corr2d_[a-z_]+)\s*\(", text))
    names = re.findall(r"\b(corr2d_[a-z_]+)\s*\(", text)
    return sorted(set(names) - inline)


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("corr2d_plan", "corr2d_homo", "corr2d_hetero", "corr2d_batched",
                     "corr2d_batched_plan", "corr2d_workspace_bytes", "corr2d_plan_destroy"):
        assert required in names
    assert sorted(B.EXPORTED) == names


def test_library_exports_every_declared_symbol():
    L = ctypes.CDLL(B.LIB_PATH)
    for name in declared_functions():
        assert hasattr(L, name), name
    out = subprocess.run(["nm", "-D", "--defined-only", B.LIB_PATH], capture_output=True,
                         text=True).stdout
    for name in declared_functions():
        assert re.search(r"\bT " + name + r"$", out, re.M), name


@pytest.mark.parametrize("lang", ["c", "c++"])
def test_header_compiles_as_c_and_cpp(tmp_path, lang):
    src = tmp_path / ("t.c" if lang == "c" else "t.cpp")
    src.write_text('#include "corr2d.h"\nint main(void){corr2d_desc d; corr2d_desc_init(&d);'
                   ' return (int)d.prec;}\n')
    cc = "gcc" if lang == "c" else "g++"
    r = subprocess.run([cc, "-std=c99" if lang == "c" else "-std=c++17", "-Wall", "-Werror",
                        "-I" + os.path.dirname(HEADER), "-c", str(src), "-o",
                        str(tmp_path / "t.o")], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr


def test_struct_layout_matches_binding():
    # offsets the ctypes mirror assumes must match the C compiler's
    prog = r'''
#include <stdio.h>
#include <stddef.h>
#include "corr2d.h"
int main(void){
 printf("%zu %zu %zu %zu %zu %zu %zu %zu %zu\n", sizeof(corr2d_desc), offsetof(corr2d_desc, norm_value),
        offsetof(corr2d_desc, tile), offsetof(corr2d_desc, scale_alpha),
        offsetof(corr2d_desc, t_in), offsetof(corr2d_desc, interp), sizeof(corr2d_item),
        sizeof(corr2d_plan_info), offsetof(corr2d_plan_info, ref1_offset));
 return 0;}
'''
    import tempfile
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "l.c")
        open(c, "w").write(prog)
        exe = os.path.join(d, "l")
        subprocess.run(["gcc", "-I" + os.path.dirname(HEADER), c, "-o", exe], check=True)
        vals = [int(x) for x in subprocess.run([exe], capture_output=True, text=True).stdout.split()]
    assert vals == [ctypes.sizeof(B.corr2d_desc), B.corr2d_desc.norm_value.offset,
                    B.corr2d_desc.tile.offset, B.corr2d_desc.scale_alpha.offset,
                    B.corr2d_desc.t_in.offset, B.corr2d_desc.interp.offset,
                    ctypes.sizeof(B.corr2d_item), ctypes.sizeof(B.corr2d_plan_info),
                    B.corr2d_plan_info.ref1_offset.offset]


def test_defaults():
    d = B.corr2d_desc_init()
    assert d.prec == B.PREC["split_bf16"] and d.basis == B.BASIS["auto"] and d.hilbert == 0
    assert d.norm_mode == 0
    assert d.in_dtype == B.DTYPE["f64"] and d.out_dtype == B.DTYPE["f32"]
    assert B.corr2d_version().startswith("corr2d")


@pytest.mark.parametrize("prec,hilbert,flags,expect", [
    ("bf16", "noda", 0, "time"), ("bf16", "circular", 0, "time"), ("bf16", "r_compat", 0, "fourier"),
    ("split_bf16", "noda", 0, "time"), ("split_f16", "noda", 0, "time"), ("f32", "noda", 0, "time"),
    ("f64", "noda", 0, "time"), ("f16", "noda", 0, "time"), ("fp8_e4m3", "noda", 0, "time"),
    ("f32", "r_compat", 0, "fourier"), ("split_bf16", "noda", B.FLAG_SPLIT_ROWS, "fourier"),
    ("split_f16", "circular", B.FLAG_SPLIT_ROWS, "fourier"),
])
def test_auto_basis_resolution(prec, hilbert, flags, expect):
    """The default basis resolves to the time basis, except with the R bin
    list and the row-selective split, which need the Fourier basis; plan
    info reports the basis in use."""
    p = B.Plan(m=64, n1=300, n2=0, prec=prec, hilbert=hilbert, flags=flags)
    assert p.info.basis == B.BASIS[expect]
    q = B.Plan(m=64, n1=300, n2=0, prec=prec, hilbert=hilbert, basis="fourier")
    assert q.info.basis == B.BASIS["fourier"]


def test_row_select_plan_workspace_and_info():
    """A row-selective plan reserves the energy partials and the selection
    record (reported by plan info); other plans report no record."""
    p = B.Plan(m=256, n1=16384, n2=0, prec="split_bf16", flags=B.FLAG_SPLIT_ROWS,
               out_layout="upper_aligned")
    q = B.Plan(m=256, n1=16384, n2=0, prec="split_bf16", out_layout="upper_aligned")
    assert q.info.sel_offset == 0
    assert p.info.sel_offset > 0 and p.info.sel_offset % 256 == 0
    assert p.info.sel_offset + 4 * 65 <= p.ws_bytes
    # energies: (n_pad/128/8) panel groups x k_pad floats for operands 0 and 2
    assert p.ws_bytes - q.ws_bytes >= 2 * 16 * 256 * 4
    h = B.Plan(m=128, n1=8192, n2=2048, prec="split_f16", flags=B.FLAG_SPLIT_ROWS)
    assert h.info.sel_offset > 0
    with pytest.raises(B.Corr2dError):
        B.Plan(B.corr2d_desc_init(prec="split_bf16", flags=B.FLAG_SPLIT_ROWS), items=[(16, 100, 0, 0, 0)])


def test_split_f16_plan_scales_per_band():
    p = B.Plan(m=256, n1=4096, n2=0, prec="split_f16")
    assert p.info.per_band_scale == 1 and p.info.k_pad == 256 and p.info.transform == 1


def _plan_status(**kw):
    base = dict(m=11, n1=512, n2=0)
    base.update(kw)
    d = B.corr2d_desc_init(**base)
    s, h = B.corr2d_plan(d, check=False)
    if h:
        B.corr2d_plan_destroy(h)
    return s


@pytest.mark.parametrize("kw,status", [
    (dict(), B.OK),
    (dict(m=1), B.EINVAL),
    (dict(m=0), B.EINVAL),
    (dict(n1=0), B.EINVAL),
    (dict(n2=-1), B.EINVAL),
    (dict(ld_in1=100), B.EINVAL),
    (dict(n2=64, ld_in2=10), B.EINVAL),
    (dict(ld_out=3), B.EINVAL),
    (dict(prec=9), B.EINVAL),
    (dict(basis=3), B.EINVAL),
    (dict(prec=7), B.EINVAL),
    (dict(prec="split_f16", flags=B.FLAG_NO_PER_BAND_SCALE), B.EUNSUPPORTED),
    (dict(hilbert=5), B.EINVAL),
    (dict(norm_mode=7), B.EINVAL),
    (dict(out_layout=3), B.EINVAL),
    (dict(in_dtype=4), B.EINVAL),
    (dict(norm_mode=2, norm_value=float("nan")), B.EINVAL),
    (dict(n2=100, out_layout=1), B.EINVAL),
    (dict(n2=100, out_layout=2), B.EINVAL),
    (dict(out_layout=2), B.OK),
    (dict(prec=5, flags=B.FLAG_NO_PER_BAND_SCALE), B.EUNSUPPORTED),
    (dict(flags=0x100), B.EINVAL),
    (dict(flags=0x40), B.EINVAL),
    (dict(flags=B.FLAG_SPLIT_ROWS), B.OK),
    (dict(flags=B.FLAG_SPLIT_ROWS, prec="split_f16"), B.OK),
    (dict(flags=B.FLAG_SPLIT_ROWS, prec="f32"), B.EUNSUPPORTED),
    (dict(flags=B.FLAG_SPLIT_ROWS, basis="time"), B.EUNSUPPORTED),
    (dict(flags=B.FLAG_SPLIT_ROWS, m=1100), B.EUNSUPPORTED),
    (dict(flags=B.FLAG_SPLIT_ROWS, m=1024), B.OK),
    (dict(split_tol=-1.0), B.EINVAL),
    (dict(split_tol=float("nan")), B.EINVAL),
    (dict(flags=B.FLAG_TRANSFORM_MATMUL), B.OK),
    (dict(tile=7), B.EINVAL),
    (dict(prec=0, tile=2), B.OK),
    (dict(prec=1, tile=3), B.EUNSUPPORTED),
    (dict(prec=2, tile=3), B.OK),
    (dict(scale_alpha=float("nan")), B.EINVAL),
    (dict(hilbert=2, basis=1), B.EUNSUPPORTED),
    (dict(hilbert=3), B.EINVAL),
    (dict(hilbert=2), B.OK),
    (dict(interp=3), B.EINVAL),
    (dict(interp=1), B.EINVAL),                                   # no t_in
    (dict(interp=1, t_in=[0.0, 1.0, 1.0, 2.0]), B.EINVAL),       # not increasing
    (dict(interp=2, t_in=[0.0, float("nan"), 2.0]), B.EINVAL),
    (dict(interp=2, t_in=[1.0]), B.EINVAL),                       # m_in = 1
    (dict(interp=2, t_in=[0.0, 0.5, 2.0, 2.2, 4.0]), B.OK),
    (dict(interp=1, t_in=[0.0, 3.0]), B.OK),
    (dict(scale_alpha=float("inf")), B.EINVAL),
    (dict(scale_alpha=0.5), B.OK),
    (dict(m=5000), B.EUNSUPPORTED),
    (dict(m=2, n1=1), B.OK),
    (dict(prec=5), B.OK),
    (dict(n2=100), B.OK),
])
def test_plan_validation(kw, status):
    assert _plan_status(**kw) == status


def test_last_error_text():
    assert _plan_status(m=1) == B.EINVAL
    assert "perturbation" in B.corr2d_last_error()


def test_workspace_bytes_monotone_in_size():
    prev = 0
    for n in (1, 100, 1000, 5000, 20000):
        d = B.corr2d_desc_init(m=64, n1=n)
        _, h = B.corr2d_plan(d)
        w = B.corr2d_workspace_bytes(h)
        assert w >= prev and w % 256 == 0
        prev = w
        B.corr2d_plan_destroy(h)


def test_plan_info():
    d = B.corr2d_desc_init(m=256, n1=16384, prec="split_bf16", out_layout="upper_packed", tile=2)
    _, h = B.corr2d_plan(d)
    info = B.corr2d_plan_get_info(h)
    assert info.k_pad == 256 and info.n_pad == 16384
    # tile 2 of the 16-bit formats: row tiles twice as tall as column tiles; the upper
    # triangle holds the tiles (I, J) with J >= 2 I
    assert (info.tile_m, info.tile_n) == (256, 128)
    t = 16384 // info.tile_m
    assert info.tiles == sum(2 * t - 2 * i for i in range(t)) == t * (t + 1)
    B.corr2d_plan_destroy(h)
    d = B.corr2d_desc_init(m=256, n1=16384, prec="split_bf16", out_layout="upper_packed", tile=3,
                           basis="fourier")
    _, h = B.corr2d_plan(d)
    info = B.corr2d_plan_get_info(h)
    assert (info.tile_m, info.tile_n) == (128, 128)
    t = 16384 // 128
    assert info.tiles == t * (t + 1) // 2
    assert info.c == pytest.approx(1.0 / (256 * 255))   # Fourier operands carry m (Parseval)
    B.corr2d_plan_destroy(h)
    d = B.corr2d_desc_init(m=256, n1=16384, prec="split_bf16", out_layout="upper_packed")
    _, h = B.corr2d_plan(d)
    assert B.corr2d_plan_get_info(h).c == pytest.approx(1.0 / 255)   # default: time basis
    B.corr2d_plan_destroy(h)
    d = B.corr2d_desc_init(m=10, n1=7, prec="f64", norm_mode="paper", basis="time")
    _, h = B.corr2d_plan(d)
    import math
    assert B.corr2d_plan_get_info(h).c == pytest.approx(10 / (math.pi * 9))
    B.corr2d_plan_destroy(h)


@pytest.mark.parametrize("kw", [dict(m=11, n1=512), dict(m=256, n1=1000, prec="f64"),
                                dict(m=64, n1=300, n2=700, prec="f32"),
                                dict(m=16, n1=300, interp="linear", t_in=np.linspace(0.0, 1.0, 9))])
def test_plan_info_reference_offsets(kw):
    """The reference spectra (n1, n2 doubles) lie inside the workspace,
    256-byte aligned, apart from each other; a homocorrelation has one."""
    _, h = B.corr2d_plan(B.corr2d_desc_init(**kw))
    info = B.corr2d_plan_get_info(h)
    ws = B.corr2d_workspace_bytes(h)
    n1, n2 = kw["n1"], kw.get("n2", 0)
    assert info.ref1_offset % 256 == 0 and info.ref1_offset + 8 * n1 <= ws
    if n2:
        assert info.ref2_offset % 256 == 0 and info.ref2_offset + 8 * n2 <= ws
        lo, hi = sorted([(info.ref1_offset, n1), (info.ref2_offset, n2)])
        assert lo[0] + 8 * lo[1] <= hi[0]
    else:
        assert info.ref2_offset == info.ref1_offset
    B.corr2d_plan_destroy(h)
    _, h = B.corr2d_batched_plan(B.corr2d_desc_init(prec="f32"), [(11, 300, 0, 0, 0)])
    info = B.corr2d_plan_get_info(h)
    assert info.ref1_offset == 0 and info.ref2_offset == 0
    B.corr2d_plan_destroy(h)


@pytest.mark.parametrize("kw,fft", [
    (dict(m=256), 1), (dict(m=128), 1), (dict(m=512), 1), (dict(m=1024), 1),
    (dict(m=64), 0), (dict(m=127), 0), (dict(m=384), 0), (dict(m=2048), 0),
    (dict(m=256, prec="f64"), 1), (dict(m=100, prec="f64"), 0), (dict(m=256, basis="time"), 1),
    (dict(m=256, basis="time", hilbert="circular"), 0),
    (dict(m=256, flags=B.FLAG_TRANSFORM_MATMUL), 0),
    (dict(m=256, hilbert="circular", basis="fourier"), 1), (dict(m=256, hilbert="r_compat"), 1),
    (dict(m=256, hilbert="circular"), 0),   # default: time basis, table product for this kernel
    (dict(m=128, n2=40), 1), (dict(m=256, prec="fp8_e4m3"), 1),
])
def test_transform_selection(kw, fft):
    """The radix FFT transform serves power-of-two 128 <= m <= 1024 (Fourier
    basis; time basis with Noda's kernel, the default), unless the flag asks
    for the product."""
    base = dict(n1=300)
    base.update(kw)
    _, h = B.corr2d_plan(B.corr2d_desc_init(**base))
    assert B.corr2d_plan_get_info(h).transform == fft
    B.corr2d_plan_destroy(h)


def test_plan_log():
    """CORR2D_LOG=1: one stderr line per plan with the decisions taken (the
    transform, tile and workspace); nothing without it."""
    import subprocess
    import sys
    code = ("from paper_1808_00685_amd import binding as B\n"
            "for kw in (dict(m=256, n1=16384, prec='split_bf16'), dict(m=11, n1=512, prec='f64')):\n"
            "    _, h = B.corr2d_plan(B.corr2d_desc_init(**kw))\n"
            "    B.corr2d_plan_destroy(h)\n"
            "items = [B.corr2d_item(m=20, n=300), B.corr2d_item(m=128, n=700, out_offset=90000)]\n"
            "_, h = B.corr2d_batched_plan(B.corr2d_desc_init(prec='f32'), items)\n"
            "B.corr2d_plan_destroy(h)\n")
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    env = dict(os.environ, CORR2D_LOG="1")
    r = subprocess.run([sys.executable, "-c", code], cwd=root, env=env, capture_output=True, text=True,
                       timeout=120)
    assert r.returncode == 0, r.stderr
    lines = [ln for ln in r.stderr.splitlines() if ln.startswith("corr2d:")]
    assert "plan split_bf16 m=256 n1=16384" in lines[0] and "transform=radix FFT" in lines[0]
    assert "plan f64 m=11 n1=512" in lines[1] and "transform=DFT table product" in lines[1]
    assert "prep_launches=2" in lines[1] and "tune:" in lines[1]
    assert "batched plan f32 items=2 distinct_m=2" in lines[2]
    assert any("persistent launch" in ln for ln in lines[3:])
    env["CORR2D_LOG"] = "0"
    r = subprocess.run([sys.executable, "-c", code], cwd=root, env=env, capture_output=True, text=True,
                       timeout=120)
    assert r.returncode == 0 and "corr2d:" not in r.stderr


def test_fused_centring_decision():
    """The table-product transform takes the centring into its own kernel for
    m <= 256 in every format but FP64, in single calls only when that launch
    has at least 512 workgroups (one per 64 spectral points and 256 transform
    rows), in batched plans whenever every set has m <= 256."""
    import subprocess
    import sys
    code = ("from paper_1808_00685_amd import binding as B\n"
            "for kw in (dict(m=200, n1=16384, prec='split_f16'), dict(m=64, n1=4096, prec='f32'),\n"
            "           dict(m=300, n1=16384, prec='split_f16'), dict(m=200, n1=16384, prec='f64'),\n"
            "           dict(m=100, n1=32768, prec='fp8_e4m3')):\n"
            "    _, h = B.corr2d_plan(B.corr2d_desc_init(**kw))\n"
            "    B.corr2d_plan_destroy(h)\n"
            "for m2 in (200, 300):\n"
            "    items = [B.corr2d_item(m=20, n=300), B.corr2d_item(m=m2, n=700, out_offset=90000)]\n"
            "    _, h = B.corr2d_batched_plan(B.corr2d_desc_init(prec='f32'), items)\n"
            "    B.corr2d_plan_destroy(h)\n")
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    env = dict(os.environ, CORR2D_LOG="1")
    r = subprocess.run([sys.executable, "-c", code], cwd=root, env=env, capture_output=True, text=True,
                       timeout=120)
    assert r.returncode == 0, r.stderr
    plans = [ln for ln in r.stderr.splitlines() if ln.startswith("corr2d: plan")]
    assert [("centring fused" in ln) for ln in plans] == [True, False, False, False, True]
    batched = [ln for ln in r.stderr.splitlines() if ln.startswith("corr2d: batched plan")]
    assert ["centring=fused" in batched[0], "centring=separate" in batched[1]] == [True, True]


def test_compute_calls_reject_bad_arguments_before_device_work():
    d = B.corr2d_desc_init(m=11, n1=64)
    _, h = B.corr2d_plan(d)
    L = B.lib()
    need = B.corr2d_workspace_bytes(h)
    fake = 1 << 20  # never dereferenced: validation fails first
    assert L.corr2d_homo(h, None, None, fake, fake, fake, need, None) == B.EINVAL
    assert L.corr2d_homo(h, fake, None, fake, fake, None, need, None) == B.EWORKSPACE
    assert L.corr2d_homo(h, fake, None, fake, fake, fake + 8, need, None) == B.EWORKSPACE
    assert L.corr2d_homo(h, fake, None, fake, fake, fake, need - 1, None) == B.EWORKSPACE
    assert L.corr2d_homo(h, fake + 1, None, fake, fake, fake, need, None) == B.EINVAL
    assert L.corr2d_hetero(h, fake, None, fake, None, fake, fake, fake, need, None) == B.EINVAL
    assert L.corr2d_batched(h, fake, fake, fake, fake, need, None) == B.EINVAL
    assert L.corr2d_homo(None, fake, None, fake, fake, fake, need, None) == B.EINVAL
    B.corr2d_plan_destroy(h)


def test_batched_plan_validation_and_sizes():
    d = B.corr2d_desc_init(prec="f32", out_layout="upper_packed")
    items = [(11, 300, 0, 0, 0), (64, 1000, 11 * 300, 0, 300 * 301 // 2)]
    _, h = B.corr2d_batched_plan(d, items)
    info = B.corr2d_plan_get_info(h)
    assert info.items == 2
    assert info.out_elements == 300 * 301 // 2 + 1000 * 1001 // 2
    B.corr2d_plan_destroy(h)
    s, h = B.corr2d_batched_plan(d, [(1, 300, 0, 0, 0)], check=False)
    assert s == B.EINVAL and not h
    s, h = B.corr2d_batched_plan(d, [(10, 300, -1, 0, 0)], check=False)
    assert s == B.EINVAL


def test_interpolation_plan_workspace_and_batched_rejected():
    base = dict(m=16, n1=300, prec="f32")
    _, h0 = B.corr2d_plan(B.corr2d_desc_init(**base))
    _, h1 = B.corr2d_plan(B.corr2d_desc_init(interp="spline", t_in=np.linspace(0.0, 1.0, 11) ** 1.5,
                                             **base))
    # resampled spectra (16 x n_pad FP64) and weights (16 x 11) live in the workspace
    assert B.corr2d_workspace_bytes(h1) >= B.corr2d_workspace_bytes(h0) + 16 * 300 * 8 + 16 * 11 * 8
    B.corr2d_plan_destroy(h0)
    B.corr2d_plan_destroy(h1)
    d = B.corr2d_desc_init(prec="f32", interp="linear", t_in=[0.0, 1.0, 3.0])
    s, _ = B.corr2d_batched_plan(d, [(3, 100, 0, 0, 0)], check=False)
    assert s == B.EUNSUPPORTED


def _aligned_layout_by_definition(n):
    """Row starts of the UPPER_ALIGNED layout from its definition: row i covers
    the columns 32 floor(i/32) .. N32-1, rows stored one after another."""
    n32 = -(-n // 32) * 32
    lens = [n32 - 32 * (i // 32) for i in range(n)]
    starts = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
    return starts, lens, n32


@pytest.mark.parametrize("n", [1, 2, 31, 32, 33, 63, 64, 65, 100, 257, 1000])
def test_upper_aligned_layout_matches_definition(n):
    starts, lens, n32 = _aligned_layout_by_definition(n)
    i, j = np.triu_indices(n)
    idx = B.upper_aligned_index(i, j, n)
    assert np.array_equal(idx, starts[i] + j - 32 * (i // 32))
    assert np.all(starts[:-1] % 32 == 0)                 # every row on a 32-element boundary
    assert len(np.unique(idx)) == len(idx)               # one slot per entry
    assert idx.min() >= 0 and idx.max() < starts[-1]
    assert B.upper_aligned_elements(n) == starts[-1] == sum(lens)
    assert B.out_elements("upper_aligned", n) == starts[-1]
    # padding bound stated in the header: at most 62 slots per row
    assert starts[-1] - n * (n + 1) // 2 <= 62 * n


def test_upper_aligned_header_helpers(tmp_path):
    # the static inline helpers of the C header against the definition
    cases = [(n, i, j) for n in (1, 33, 100, 16384, 70001) for i, j in
             ((0, 0), (0, n - 1), (n // 3, n // 2), (n - 1, n - 1), (min(31, n - 1), n - 1))]
    prog = "#include <stdio.h>\n#include \"corr2d.h\"\nint main(void){\n"
    for n, i, j in cases:
        prog += f'printf("%lld\\n", (long long)corr2d_upper_aligned_index({i}, {j}, {n}));\n'
    for n in (1, 33, 100, 16384, 70001):
        prog += f'printf("%lld\\n", (long long)corr2d_upper_aligned_elements({n}));\n'
    prog += "return 0;}\n"
    c = tmp_path / "a.c"
    c.write_text(prog)
    exe = tmp_path / "a"
    subprocess.run(["gcc", "-std=c99", "-Wall", "-Werror", "-I" + os.path.dirname(HEADER), str(c),
                    "-o", str(exe)], check=True)
    got = [int(x) for x in subprocess.run([str(exe)], capture_output=True, text=True).stdout.split()]
    want = []
    for n, i, j in cases:
        n32 = -(-n // 32) * 32
        start = sum(n32 - 32 * (k // 32) for k in range(i))
        want.append(start + j - 32 * (i // 32))
    for n in (1, 33, 100, 16384, 70001):
        n32 = -(-n // 32) * 32
        want.append(sum(n32 - 32 * (k // 32) for k in range(n)))
    assert got == want


def test_batched_out_elements_upper_aligned():
    d = B.corr2d_desc_init(prec="f32", out_layout="upper_aligned")
    e300 = B.upper_aligned_elements(300)
    items = [(11, 300, 0, 0, 0), (64, 1000, 11 * 300, 0, e300)]
    _, h = B.corr2d_batched_plan(d, items)
    assert B.corr2d_plan_get_info(h).out_elements == e300 + B.upper_aligned_elements(1000)
    B.corr2d_plan_destroy(h)


def test_result_object_argument_errors_before_any_call():
    """corr2d() and hetero() reject inconsistent arguments before a plan is
    made or any device memory is touched (CPU tensors suffice)."""
    import torch
    y = torch.zeros(8, 10, dtype=torch.float64)
    with pytest.raises(ValueError):
        B.corr2d(y, ref2=y[0])
    with pytest.raises(ValueError):
        B.corr2d(y, wave2=torch.arange(10.0))
    with pytest.raises(ValueError):
        B.corr2d(y, y, layout="upper_aligned")
    with pytest.raises(ValueError):
        B.hetero(y, torch.zeros(9, 10, dtype=torch.float64))


def test_noalloc_scratch_size_matches_header(tmp_path):
    src = tmp_path / "s.c"
    src.write_text('#include <stdio.h>\n#include "corr2d.h"\n'
                   'int main(void){printf("%zu\\n", CORR2D_NOALLOC_SCRATCH_BYTES); return 0;}\n')
    exe = tmp_path / "s"
    r = subprocess.run(["gcc", "-I" + os.path.dirname(HEADER), str(src), "-o", str(exe)],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    assert int(subprocess.run([str(exe)], capture_output=True, text=True).stdout) == \
        B.NOALLOC_SCRATCH_BYTES


def test_noalloc_rejects_before_device_work():
    """The allocation-free entry point checks the plan before any HIP call:
    a NULL plan, a heterocorrelation or batched plan, an interpolation plan,
    and a plan whose workspace exceeds the fixed scratch."""
    L = B.lib()
    st = L.corr2d_homo_noalloc(None, None, None, None, None, None)
    assert st == B.EINVAL
    het = B.Plan(m=16, n1=64, n2=32, prec="f32")
    assert B.corr2d_homo_noalloc(het.handle, 1, None, 1, 1, check=False) == B.EINVAL
    it = B.Plan(m=8, n1=64, n2=0, prec="f32", t_in=np.linspace(0.0, 1.0, 9) ** 2, interp="linear")
    assert B.corr2d_homo_noalloc(it.handle, 1, None, 1, 1, check=False) == B.EUNSUPPORTED
    big = B.Plan(m=256, n1=16384, n2=0, prec="f64", out_layout="upper_aligned", out_dtype="f64")
    assert big.ws_bytes > B.NOALLOC_SCRATCH_BYTES
    assert B.corr2d_homo_noalloc(big.handle, 1, None, 1, 1, check=False) == B.EWORKSPACE
    assert b"fixed scratch" in L.corr2d_last_error()
    fits = B.Plan(m=256, n1=16384, n2=0, prec="split_bf16", out_layout="upper_aligned")
    assert fits.ws_bytes <= B.NOALLOC_SCRATCH_BYTES


def test_batched_plan_one_tile_shape():
    """A batched plan runs every data set in one tile shape, the tuned shape
    of the set with the largest m n^2, so its contraction is one persistent
    launch even where single calls of its sets would take different shapes."""
    import subprocess
    import sys
    code = ("from paper_1808_00685_amd import binding as B\n"
            "for kw in (dict(m=20, n1=300, prec='f32'), dict(m=128, n1=16000, prec='f32')):\n"
            "    _, h = B.corr2d_plan(B.corr2d_desc_init(**kw))\n"
            "    print('single', B.corr2d_plan_get_info(h).tile)\n"
            "    B.corr2d_plan_destroy(h)\n"
            "items = [B.corr2d_item(m=20, n=300), B.corr2d_item(m=128, n=16000, out_offset=90000)]\n"
            "_, h = B.corr2d_batched_plan(B.corr2d_desc_init(prec='f32'), items)\n"
            "B.corr2d_plan_destroy(h)\n")
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    env = dict(os.environ, CORR2D_LOG="1")
    r = subprocess.run([sys.executable, "-c", code], cwd=root, env=env, capture_output=True, text=True,
                       timeout=120)
    assert r.returncode == 0, r.stderr
    singles = [int(ln.split()[1]) for ln in r.stdout.splitlines() if ln.startswith("single")]
    assert len(set(singles)) == 2
    launches = [ln for ln in r.stderr.splitlines() if "one persistent launch" in ln]
    assert len(launches) == 1
    assert f"tile {singles[1]} " in launches[0] and "2 data sets" in launches[0]
