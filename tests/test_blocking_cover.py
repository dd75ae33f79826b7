"""Host-side model of the fused red+black sweep's tile (temporal blocking):
for every tile of a range of level shapes and boundary conditions, each tile
element that the black half-sweep of the tile's cells reads must, after the
red pass over the widened region and the refresh of the wall images, hold the
value the plain red half-sweep would give it (a red source cell relaxed, a
face written by the red cell next to it), and every access must stay inside
the widened tile.  Index logic only; the arithmetic is checked on the GPU
against the oracle."""
import pytest

TX = TY = 16
W, H = TX + 7, TY + 7


def _wrap(k, n):
    return k + n if k < 0 else (k - n if k >= n else k)


def _check(m1, m2, bcx, bcy):
    nt = 0
    for j0 in range(0, m2, TY):
        for i0 in range(0, m1, TX):
            nt += 1
            ti0, tj0 = i0 - 2, j0 - 2  # tile origin: positions ti0-1 .. ti0+W-2

            def inside(i, j):
                return ti0 - 1 <= i <= ti0 + W - 2 and tj0 - 1 <= j <= tj0 + H - 2

            def real(i, j):
                return (bcx or 0 <= i < m1) and (bcy or 0 <= j < m2)

            # red pass: cells i+j even of the widened region, real ones only
            red = set()
            for tj in range(j0 - 2, j0 + TY + 2):
                for ti in range(i0 - 2, i0 + TX + 2):
                    if (ti + tj) % 2 == 0 and real(ti, tj):
                        # its stencil (cells -1..+1, faces up to +2) stays in the tile
                        for dj in (-1, 0, 1, 2):
                            for di in (-1, 0, 1, 2):
                                assert inside(ti + di, tj + dj), (m1, m2, i0, j0, ti, tj)
                        red.add((ti, tj))
            # faces written by the red pass (lo face of the cell, hi face of the
            # cell when it is an unknown)
            uw, vw = set(), set()
            for (ti, tj) in red:
                i, j = _wrap(ti, m1) if bcx else ti, _wrap(tj, m2) if bcy else tj
                if bcx or i >= 1:
                    uw.add((ti, tj))
                if bcx or i + 1 < m1:
                    uw.add((ti + 1, tj))
                if bcy or j >= 1:
                    vw.add((ti, tj))
                if bcy or j + 1 < m2:
                    vw.add((ti, tj + 1))
            # every element the black cells of the tile read
            for j in range(j0 - 1, j0 + TY + 2):
                for i in range(i0 - 1, i0 + TX + 2):
                    if (not bcx and i > m1 + 1) or (not bcy and j > m2 + 1):
                        continue  # beyond the reach of any cell
                    assert inside(i, j)
                    gx = not bcx and (i < 0 or i >= m1)
                    gy = not bcy and (j < 0 or j >= m2)
                    si = (0 if i < 0 else m1 - 1) if gx else i
                    sj = (0 if j < 0 else m2 - 1) if gy else j
                    # cell fields: the source cell's value after the red pass
                    if (si + sj) % 2 == 0:
                        assert (si, sj) in red, ("cell", m1, m2, bcx, bcy, i0, j0, i, j)
                    # u face: zero on or beyond an x wall, else written by a red
                    # cell (reflected from the wall row across a y wall)
                    if bcx or 0 < i < m1:
                        assert (i, sj) in uw, ("u", m1, m2, bcx, bcy, i0, j0, i, j)
                    if bcy or 0 < j < m2:
                        assert (si, j) in vw, ("v", m1, m2, bcx, bcy, i0, j0, i, j)
    return nt


@pytest.mark.parametrize("m1,m2", [(32, 64), (64, 32), (48, 80), (40, 24), (128, 256)])
@pytest.mark.parametrize("bcx,bcy", [(0, 0), (1, 0), (0, 1), (1, 1)])
def test_fused_tile_reads_post_red_values(m1, m2, bcx, bcy):
    if (bcx and m1 < TX + 3) or (bcy and m2 < TY + 3):
        pytest.skip("periodic axis too short for a single wrap: those levels keep the half-sweeps")
    assert _check(m1, m2, bcx, bcy) > 0


def test_region_fits_the_workgroup():
    # lane pairs of the widened red region and of the tile's black cells
    assert (TX + 4) * (TY + 4) <= 2 * TX * TY
    assert 14 * W * H * 8 <= 65536
