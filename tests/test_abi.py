"""The C-ABI library: it loads, exports every declared symbol, and rejects bad
arguments on the host (no GPU needed: validation runs before any HIP call)."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "hyres.h")


def _lib():
    from paper_2204_06979_amd import _lib as L
    try:
        return L, L.lib()
    except ImportError as e:  # pragma: no cover
        pytest.skip(str(e))


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(hyres_[a-z0-9_]+)\s*\(", text)))


def test_every_declared_symbol_is_exported():
    L, lib = _lib()
    names = declared_functions()
    assert len(names) >= 15
    for n in names:
        assert hasattr(lib, n), n
    # and the binding declares them all
    for n in names:
        assert n in L.SIGNATURES, n


def test_status_strings_and_coeff_count():
    L, lib = _lib()
    assert lib.hyres_status_string(0) == b"ok"
    assert b"shape" in lib.hyres_status_string(2)
    assert lib.hyres_coeff_count(349, 1905, 4) == 668361
    assert lib.hyres_coeff_count(64, 64, 3) == 4096
    assert lib.hyres_coeff_count(3, 64, 1) == 0          # level input shorter than the filter
    assert lib.hyres_coeff_count(64, 64, 9) == 0         # too many levels


def test_workspace_sizes_and_shape_errors():
    L, lib = _lib()
    nb = C.c_size_t()
    opt = L.Options(8, 4, L.PREC_NATIVE, L.SCOPE_ALL)
    assert lib.hyres_denoise_workspace_size(349, 1905, 144, C.byref(opt), L.HYRES_F32, C.byref(nb)) == 0
    big = nb.value
    assert 50e6 < big < 120e6
    assert lib.hyres_denoise_workspace_size(64, 64, 32, C.byref(L.Options(4, 3, 0, 0)), L.HYRES_F64,
                                            C.byref(nb)) == 0
    assert nb.value < big
    bad = [L.Options(0, 4, 0, 0), L.Options(17, 4, 0, 0), L.Options(8, 0, 0, 0), L.Options(8, 9, 0, 0),
           L.Options(8, 4, 0, 5)]
    for o in bad:
        assert lib.hyres_denoise_workspace_size(349, 1905, 144, C.byref(o), L.HYRES_F32, C.byref(nb)) == 2
    assert lib.hyres_denoise_workspace_size(349, 1905, 144, C.byref(opt), 7, C.byref(nb)) == 3
    assert lib.hyres_denoise_workspace_size(349, 1905, 1, C.byref(L.Options(1, 4, 0, 0)), 0, C.byref(nb)) == 2
    assert lib.hyres_denoise_workspace_size(349, 1905, 300, C.byref(opt), 0, C.byref(nb)) == 2
    # mixed precision needs an FP32 cube
    assert lib.hyres_denoise_workspace_size(64, 64, 32, C.byref(L.Options(4, 3, 1, 0)), L.HYRES_F64,
                                            C.byref(nb)) == 3
    assert lib.hyres_denoise_workspace_size(64, 64, 32, C.byref(L.Options(4, 3, 1, 0)), L.HYRES_F32,
                                            C.byref(nb)) == 0
    assert lib.hyres_dwt2_workspace_size(4, 5, 64, 2, 0, C.byref(nb)) == 2   # 5 -> 3 < 4 at level 2
    assert lib.hyres_dwt2_workspace_size(4, 64, 64, 3, 0, C.byref(nb)) == 0
    assert lib.hyres_sure_workspace_size(0, 100, 0, C.byref(nb)) == 2
    assert lib.hyres_sure_workspace_size(3, 100, 0, C.byref(nb)) == 0


def test_entry_points_reject_bad_arguments_before_touching_the_device():
    L, lib = _lib()
    fake = C.create_string_buffer(64)           # never dereferenced on these paths
    h = C.cast(fake, C.c_void_p)
    opt = L.Options(4, 3, 0, 0)
    ws = C.create_string_buffer(1 << 12)
    wsp = C.cast(ws, C.c_void_p).value
    wsp_al = (wsp + 255) // 256 * 256
    # NULL handle / cube
    assert lib.hyres_denoise(None, wsp, 64, 64, 32, 32, 2048, 0, C.byref(opt), None, None, wsp, 32, 2048,
                             None, wsp_al, 100, None) == 1
    assert lib.hyres_denoise(h, None, 64, 64, 32, 32, 2048, 0, C.byref(opt), None, None, wsp, 32, 2048,
                             None, wsp_al, 100, None) == 1
    # pitch smaller than p
    assert lib.hyres_denoise(h, wsp, 64, 64, 32, 16, 2048, 0, C.byref(opt), None, None, wsp, 32, 2048,
                             None, wsp_al, 100, None) == 2
    # row pitch too small
    assert lib.hyres_denoise(h, wsp, 64, 64, 32, 32, 100, 0, C.byref(opt), None, None, wsp, 32, 2048,
                             None, wsp_al, 100, None) == 2
    # rank > 16
    assert lib.hyres_denoise(h, wsp, 64, 64, 32, 32, 2048, 0, C.byref(L.Options(17, 3, 0, 0)), None, None,
                             wsp, 32, 2048, None, wsp_al, 100, None) == 2
    # workspace too small, and misaligned
    assert lib.hyres_denoise(h, wsp, 64, 64, 32, 32, 2048, 0, C.byref(opt), None, None, wsp, 32, 2048,
                             None, wsp_al, 100, None) == 4
    assert lib.hyres_denoise(h, wsp, 64, 64, 32, 32, 2048, 0, C.byref(opt), None, None, wsp, 32, 2048,
                             None, wsp_al + 8, 1 << 40, None) == 4
    # SURE with stride < Nc
    assert lib.hyres_sure_threshold(h, wsp, 2, 100, 50, 0, wsp, None, None, wsp_al, 1 << 40, None) == 2
    # estimate_noise requires sigma_out
    assert lib.hyres_estimate_noise(h, wsp, 8, 8, 4, 4, 32, 0, None, None, None, wsp_al, 1 << 20, None) == 1


def test_tile_grid_matches_the_generator_rule():
    from paper_2204_06979_amd import synth
    L, lib = _lib()
    n = C.c_int()
    buf = (C.c_int * 64)()
    for size, tile, ov in [(2048, 512, 32), (1000, 512, 32), (512, 512, 32), (300, 512, 32), (260, 128, 16),
                           (129, 64, 0), (4096, 256, 64)]:
        assert lib.hyres_tile_grid(size, tile, ov, buf, C.byref(n)) == 0
        assert [buf[i] for i in range(n.value)] == synth.tile_starts(size, tile, ov), (size, tile, ov)
    assert lib.hyres_tile_grid(2048, 512, 300, buf, C.byref(n)) == 2      # overlap > tile / 2
    assert lib.hyres_tile_grid(100000, 64, 0, buf, C.byref(n)) == 6       # more than 64 tiles
    nb = C.c_size_t()
    opt = L.Options(10, 4, L.PREC_MIXED, L.SCOPE_ALL)
    assert lib.hyres_tiled_workspace_size(2048, 2048, 224, 512, 32, C.byref(opt), L.HYRES_F32, C.byref(nb)) == 0
    per_tile = C.c_size_t()
    assert lib.hyres_denoise_workspace_size(512, 512, 224, C.byref(opt), L.HYRES_F32, C.byref(per_tile)) == 0
    assert 25 * per_tile.value * 0.9 < nb.value < 25 * per_tile.value * 1.1
    # a tile too small for the levels
    assert lib.hyres_tiled_workspace_size(256, 256, 32, 16, 4, C.byref(opt), L.HYRES_F32, C.byref(nb)) == 2


def test_batch_workspace_and_validation():
    L, lib = _lib()
    nb = C.c_size_t()
    opt = L.Options(0, 0, L.PREC_MIXED, L.SCOPE_ALL)
    cubes = (L.Cube * 3)()
    for i, (H, W, p, r, lv) in enumerate([(128, 200, 103, 6, 4), (300, 129, 224, 12, 4), (64, 64, 32, 4, 3)]):
        cubes[i].H, cubes[i].W, cubes[i].p, cubes[i].rank, cubes[i].levels = H, W, p, r, lv
    assert lib.hyres_batch_workspace_size(cubes, 3, L.HYRES_F32, C.byref(opt), C.byref(nb)) == 0
    total = 0
    for i in range(3):
        one = C.c_size_t()
        o = L.Options(cubes[i].rank, cubes[i].levels, L.PREC_MIXED, L.SCOPE_ALL)
        assert lib.hyres_denoise_workspace_size(cubes[i].H, cubes[i].W, cubes[i].p, C.byref(o), L.HYRES_F32,
                                                C.byref(one)) == 0
        total += one.value
    assert total * 0.9 < nb.value < total * 1.1
    cubes[1].rank = 17
    assert lib.hyres_batch_workspace_size(cubes, 3, L.HYRES_F32, C.byref(opt), C.byref(nb)) == 2
    cubes[1].rank = 12
    assert lib.hyres_batch_workspace_size(cubes, 3, L.HYRES_F64, C.byref(opt), C.byref(nb)) == 3   # mixed needs F32
    assert lib.hyres_batch_workspace_size(cubes, 0, L.HYRES_F32, C.byref(opt), C.byref(nb)) == 2
    # creation rejects missing cube pointers before touching the device
    fake = C.create_string_buffer(64)
    bp = C.c_void_p()
    assert lib.hyres_batch_create(C.cast(fake, C.c_void_p), cubes, 3, L.HYRES_F32, C.byref(opt), None, 0, None,
                                  C.byref(bp)) == 1


def test_rank_flags_validation():
    """Both rank rules at once, and a data-chosen rank with the adjoint, are refused."""
    L, lib = _lib()
    nb = C.c_size_t()
    for f in (L.FLAG_RANK_HYSIME, L.FLAG_RANK_SURE):
        assert lib.hyres_denoise_workspace_size(64, 64, 32, C.byref(L.Options(8, 3, 0, 0, f)), L.HYRES_F32,
                                                C.byref(nb)) == 0
        assert lib.hyres_denoise_backward_workspace_size(64, 64, 32, C.byref(L.Options(8, 3, 0, 0, f)),
                                                         L.HYRES_F32, C.byref(nb)) == 6
    both = L.Options(8, 3, 0, 0, L.FLAG_RANK_HYSIME | L.FLAG_RANK_SURE)
    assert lib.hyres_denoise_workspace_size(64, 64, 32, C.byref(both), L.HYRES_F32, C.byref(nb)) == 6


def test_method_workspace_validation():
    """WSRRR takes native precision and a given rank only; FORPDN's workspace
    grows with the levels and shrinks when sigma is given; bad shapes are refused."""
    L, lib = _lib()
    nb = C.c_size_t()
    assert lib.hyres_wsrrr_workspace_size(64, 64, 32, C.byref(L.Options(4, 3, L.PREC_NATIVE, 0, 0)), L.HYRES_F32,
                                          C.byref(nb)) == 0
    assert nb.value > 0
    assert lib.hyres_wsrrr_workspace_size(64, 64, 32, C.byref(L.Options(4, 3, L.PREC_MIXED, 0, 0)), L.HYRES_F32,
                                          C.byref(nb)) == 6
    assert lib.hyres_wsrrr_workspace_size(64, 64, 32, C.byref(L.Options(4, 3, 0, 0, L.FLAG_RANK_SURE)),
                                          L.HYRES_F32, C.byref(nb)) == 6
    sizes = []
    for given in (0, 1):
        assert lib.hyres_forpdn_workspace_size(64, 64, 32, 3, L.HYRES_F32, given, C.byref(nb)) == 0
        sizes.append(nb.value)
    assert sizes[1] < sizes[0]
    assert lib.hyres_forpdn_workspace_size(64, 64, 32, 0, L.HYRES_F32, 0, C.byref(nb)) == 2
    assert lib.hyres_forpdn_workspace_size(6, 64, 32, 2, L.HYRES_F32, 0, C.byref(nb)) == 2    # level 2 below 4 x 4
    assert lib.hyres_forpdn_workspace_size(64, 64, 1, 2, L.HYRES_F32, 0, C.byref(nb)) == 2
