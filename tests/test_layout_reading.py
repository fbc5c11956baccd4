"""CPU checks of the paper's sliced-layout transformation (Sec. 2), as the layout
kernels read it: x' = x, y' = y - x, z' = x - y + z (mod L) is a bijection of the periodic
cube, every z' plane holds sites of one colour, and each site's six neighbours sit
at the transformed offsets the paper lists, three in the plane above and three in
the plane below.  These are properties of the transformation itself, checked by
enumeration; the GPU layout tests check the kernel that uses them."""
import numpy as np
import pytest


def transform(L, x, y, z):
    return x % L, (y - x) % L, (x - y + z) % L


def inverse(L, xp, yp, zp):
    return xp % L, (yp + xp) % L, (zp + yp) % L


@pytest.mark.parametrize("L", [2, 4, 6, 8, 10])
def test_transformation_is_a_bijection_with_its_inverse(L):
    z, y, x = np.meshgrid(np.arange(L), np.arange(L), np.arange(L), indexing="ij")
    xp, yp, zp = transform(L, x, y, z)
    idx = xp + L * (yp + L * zp)
    assert np.unique(idx).size == L**3
    bx, by, bz = inverse(L, xp, yp, zp)
    assert np.array_equal(bx, x) and np.array_equal(by, y) and np.array_equal(bz, z)


@pytest.mark.parametrize("L", [2, 4, 6, 8, 10])
def test_every_transformed_plane_has_one_colour(L):
    z, y, x = np.meshgrid(np.arange(L), np.arange(L), np.arange(L), indexing="ij")
    _, _, zp = transform(L, x, y, z)
    colour = (x + y + z) & 1
    for p in range(L):
        cols = np.unique(colour[zp == p])
        assert cols.size == 1 and cols[0] == p & 1  # red (x+y+z even) on even planes


# neighbour of the cube site -> offset (dx', dy', dz') in transformed coordinates
NEIGHBOURS = {
    (0, 0, +1): (0, 0, +1),    # +z
    (0, -1, 0): (0, -1, +1),   # -y
    (+1, 0, 0): (+1, -1, +1),  # +x
    (0, 0, -1): (0, 0, -1),    # -z
    (0, +1, 0): (0, +1, -1),   # +y
    (-1, 0, 0): (-1, +1, -1),  # -x
}


@pytest.mark.parametrize("L", [2, 4, 6, 8])
def test_neighbours_sit_at_the_listed_offsets(L):
    for x in range(L):
        for y in range(L):
            for z in range(L):
                xp, yp, zp = transform(L, x, y, z)
                for (dx, dy, dz), (ex, ey, ez) in NEIGHBOURS.items():
                    want = transform(L, x + dx, y + dy, z + dz)
                    got = ((xp + ex) % L, (yp + ey) % L, (zp + ez) % L)
                    assert got == want, (L, (x, y, z), (dx, dy, dz))


def test_plane_index_per_colour():
    """With planes numbered per colour (m = z'/2), a red site of plane m reads the
    blue planes m and m - 1; a blue site of plane m reads the red planes m + 1 and m
    (wrapping over L/2 planes)."""
    L = 8
    M = L // 2
    for zp in range(L):
        c, m = zp & 1, zp // 2
        up, down = (zp + 1) % L, (zp - 1) % L
        assert up & 1 != c and down & 1 != c
        assert up // 2 == (m + c) % M
        assert down // 2 == (m + c - 1) % M
