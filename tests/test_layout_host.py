"""Host-side checks of the column-blocked layout the kernels use for the
W_c-basis vectors (Tq, Tv, T): element (row, c) lives at
((c / B) rows + row) B + c % B.  The contiguous-axis passes reach it in the
blocked lane order (W consecutive positions, row, next W positions; W = 16
FP64 or 32 FP32 entries) and the strided passes through their tile base /
stride; both must visit every element exactly once, agree on its
address, and stay inside the rows x (n_last + 63) allocation for every block
width B <= 64 the tiler can choose.  Pure index arithmetic, no GPU.
"""
import pytest


def _ilog2(v):
    return v.bit_length() - 1


def _check(shape, B, lp_row):
    d = len(shape)
    n = list(shape) + [1] * (3 - d)
    nlast = shape[-1]
    rows = 1
    for k in range(d - 1):
        rows *= shape[k]
    lgB = _ilog2(B)
    qblk = rows << lgB
    cap = rows * (nlast + 63)

    def addr(row, c):
        return ((c >> lgB) * rows + row) * B + (c & (B - 1))

    # contiguous-axis tiles, blocked lane order
    lgl = _ilog2(lp_row)
    for lgW in (4, 5):
        seen = set()
        for tile in range((rows + lp_row - 1) // lp_row):
            row0 = tile * lp_row
            nl = min(lp_row, rows - row0)
            total = ((nlast + (1 << lgW) - 1) >> lgW) << (lgW + lgl)
            for e in range(total):
                rl = e & ((1 << lgW) - 1)
                l = (e >> lgW) & (lp_row - 1)
                r = ((e >> (lgW + lgl)) << lgW) + rl
                q = (r >> lgB) * qblk + (row0 << lgB) + (l << lgB) + (r & (B - 1))
                if l < nl and r < nlast:
                    assert q == addr(row0 + l, r) and 0 <= q < cap
                    assert (row0 + l, r) not in seen
                    seen.add((row0 + l, r))
        assert len(seen) == rows * nlast
    # strided tiles (lines = one block) along every non-contiguous axis
    for ax in range(d - 1):
        nblk = (nlast + B - 1) // B
        nouter = 1 if d == 2 else (n[1] if ax == 0 else n[0])
        seen = set()
        for tile in range(nouter * nblk):
            outer, blk = divmod(tile, nblk)
            c0 = blk * B
            nl = min(B, nlast - c0)
            rbase, rstep = 0, 1
            if d == 3:
                if ax == 1:
                    rbase = outer * n[1]
                else:
                    rbase, rstep = outer, n[1]
            base = (blk * rows + rbase) << lgB
            stride = rstep << lgB
            for r in range(shape[ax]):
                for l in range(nl):
                    p = base + l + r * stride
                    if d == 2:
                        row = r
                    elif ax == 0:
                        row = r * n[1] + outer
                    else:
                        row = outer * n[1] + r
                    assert p == addr(row, c0 + l) and 0 <= p < cap
                    seen.add((row, c0 + l))
        assert len(seen) == rows * nlast


@pytest.mark.parametrize("shape", [(7, 7), (15, 31), (63, 63), (3, 511), (127, 255),
                                   (1023, 7), (7, 15, 31), (31, 31, 31), (15, 63, 127)])
def test_blocked_layout_maps(shape):
    nlast = shape[-1]
    for B in [1, 2, 4, 8, 16, 32, 64]:
        if B > 2 * (1 << _ilog2(nlast)):
            continue
        for lp_row in [1, 2, 4, 8]:
            _check(shape, B, lp_row)
