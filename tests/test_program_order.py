"""Stream order of the launch programs, checked on the host (no GPU needed).

A batch or tile grid runs its cubes in groups on side streams forked from and
joined back into the caller's stream.  The library walks the program it would
enqueue without touching a device (hyres_batch_check_program,
hyres_tiled_check_program) and checks that every wait on an event follows a
record of that event in the same program, and that every side stream starts
with a wait and ends joined into the caller's stream.  Here that is checked
for every grouping the planner can produce: one to five small-solve classes
(groups are capped at four), cubes with and without given thresholds, both
element types and precisions, and tile grids of one to many tiles.
"""
import ctypes as C
import itertools

import pytest


def _lib():
    from paper_2204_06979_amd import _lib as L
    try:
        return L, L.lib()
    except ImportError as e:  # pragma: no cover
        pytest.skip(str(e))


# one band count per small-solve class (the classes end at 32, 64, 96, 128,
# 144, 160, 176, 192, 224 bands)
CLASS_P = [24, 60, 90, 120, 140, 150, 170, 190, 220]


def _cubes(L, ps, with_lambda=()):
    arr = (L.Cube * len(ps))()
    keep = []
    for i, p in enumerate(ps):
        H, W = 64 + 8 * i, 96 - 4 * i
        lam = None
        if i in with_lambda:
            lam = C.c_void_p(0x1000)          # never dereferenced by the check
            keep.append(lam)
        arr[i] = L.Cube(None, H, W, p, p, W * p, None, p, W * p, min(4, p - 1), 3, None,
                        lam.value if lam else None, L.Outputs())
    return arr, keep


@pytest.mark.parametrize("nclass", [1, 2, 3, 4, 5, 9])
@pytest.mark.parametrize("dtype,prec", [(0, 0), (0, 1), (1, 0)])
def test_batch_programs_record_before_wait(nclass, dtype, prec):
    L, lib = _lib()
    for classes in itertools.islice(itertools.combinations(range(9), nclass), 6):
        ps = [CLASS_P[c] for c in classes]
        ps = ps + ps[::-1]                     # two cubes per class, mixed order
        for with_lambda in ((), (0,), tuple(range(len(ps)))):
            arr, keep = _cubes(L, ps, with_lambda)
            st = L.ProgramStats()
            opt = L.Options(0, 0, prec, 0, 0)
            rc = lib.hyres_batch_check_program(arr, len(ps), dtype, C.byref(opt), C.byref(st))
            assert rc == 0, (classes, with_lambda, rc)
            assert st.groups == min(nclass, 4)
            assert st.streams == st.groups
            assert st.launches > 0
            # one fork wait per side stream, one chain wait per later group, one join wait per side stream
            assert st.waits == 3 * (st.groups - 1)


@pytest.mark.parametrize("H,W,p,tile,ov", [(64, 64, 32, 64, 8), (200, 130, 64, 64, 8), (300, 260, 40, 128, 16),
                                           (2048, 2048, 224, 512, 32), (97, 300, 17, 128, 32),
                                           (1000, 90, 103, 96, 16)])
@pytest.mark.parametrize("dtype,prec", [(0, 0), (0, 1), (1, 0)])
def test_tiled_programs_record_before_wait(H, W, p, tile, ov, dtype, prec):
    L, lib = _lib()
    st = L.ProgramStats()
    opt = L.Options(min(4, p - 1), 2, prec, 0, 0)
    rc = lib.hyres_tiled_check_program(H, W, p, tile, ov, C.byref(opt), dtype, C.byref(st))
    assert rc == 0, rc
    ntiles = len(range(0, 1)) if tile >= H and tile >= W else None
    assert st.groups >= 1 and st.groups <= 4
    assert st.streams == st.groups
    assert st.waits == 3 * (st.groups - 1)
    if ntiles == 1:
        assert st.groups == 1


def test_check_rejects_what_create_rejects():
    L, lib = _lib()
    arr, _ = _cubes(L, [300])                  # more than 224 bands
    st = L.ProgramStats()
    assert lib.hyres_batch_check_program(arr, 1, 0, C.byref(L.Options(0, 0, 0, 0, 0)), C.byref(st)) == 2
    assert lib.hyres_tiled_check_program(64, 64, 32, 64, 40, C.byref(L.Options(4, 2, 0, 0, 0)), 0,
                                         C.byref(st)) == 2
