"""Host-side check of the LDS slot layout of pass 1's gate cell sums (no
GPU).  Each pass-1 tile keeps one LDS slot per (cell row, cell column) index
it spans, indexed from its first cell; the host sizes the slots with

    slots = min(CX, floor((TW - 1) CX / W) + 2)
    crows = min(CY, floor((rows - 1) CY / H) + 2)

(column x lies in cell floor(x CX / W), row y in floor(y CY / H)).  A slot
index past these would write outside the tile's LDS slots, so every tile of
every shape below is walked and its spans compared with the bounds: the
bound holds because floor(a) - floor(b) <= floor(a - b) + 1, and the cell
indices stay below CX and CY."""
import numpy as np

TW = 248            # output columns of a pass-1 tile (4 waves x 62)
CELLS = 128


def bounds(W, H, rows, gx=1, gy=1):
    CX, CY = CELLS * gx, CELLS * gy
    return min(CX, (TW - 1) * CX // W + 2), min(CY, (rows - 1) * CY // H + 2)


def spans(W, H, rows, gx=1, gy=1):
    CX, CY = CELLS * gx, CELLS * gy
    sx = max((min(x0 + TW, W) - 1) * CX // W - x0 * CX // W + 1 for x0 in range(0, W, TW))
    sy = max((min(y0 + rows, H) - 1) * CY // H - y0 * CY // H + 1 for y0 in range(0, H, rows))
    return sx, sy


def test_slot_bounds_cover_every_tile():
    rng = np.random.default_rng(8)
    shapes = [(1, 1, 64), (77, 100, 38), (100, 77, 64), (9, 180000, 64), (180000, 9, 64), (2048, 2048, 64),
              (127, 129, 1), (128, 128, 1024), (249, 250, 7), (16384, 16384, 64)]
    shapes += [(int(rng.integers(1, 5000)), int(rng.integers(1, 5000)), int(rng.integers(1, 200)))
               for _ in range(300)]
    for W, H, rows in shapes:
        for g in (1, 2, 4):
            if g > 1 and (W % g or H % g):
                continue
            bs, br = bounds(W, H, rows, g, g)
            ss, sr = spans(W, H, rows, g, g)
            assert ss <= bs and sr <= br, (W, H, rows, g, ss, bs, sr, br)


def test_bounds_are_tight_somewhere():
    # the +2 is reached: a tile straddling cells at both ends
    assert spans(1000, 64, 64)[0] == bounds(1000, 64, 64)[0]
