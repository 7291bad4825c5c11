"""CPU checks of the benchmark's algorithmic byte counts (the numerators of
its roofline figures), against closed forms and brute force."""
import itertools
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import bench  # noqa: E402


def brute_ras(nx, ny, nz, parts, ov):
    """Sum over subdomains of |Omega_s| and of the lower neighbour pairs inside
    Omega_s, by enumerating every cell (Omega_s: cells within graph distance
    ov of the box; boxes split the axes with the first n mod p one longer)."""
    def bounds(n, p):
        base, rem = divmod(n, p)
        out, a = [], 0
        for b in range(p):
            w = base + (1 if b < rem else 0)
            out.append((a, a + w))
            a += w
        return out

    cells = pairs = 0
    for bx, by, bz in itertools.product(bounds(nx, parts[0]), bounds(ny, parts[1]), bounds(nz, parts[2])):
        def dist(v, b):
            return b[0] - v if v < b[0] else (v - b[1] + 1 if v >= b[1] else 0)

        inside = {(i, j, k) for i in range(nx) for j in range(ny) for k in range(nz)
                  if dist(i, bx) + dist(j, by) + dist(k, bz) <= ov}
        cells += len(inside)
        pairs += sum(((i - 1, j, k) in inside) + ((i, j - 1, k) in inside) + ((i, j, k - 1) in inside)
                     for (i, j, k) in inside)
    return cells, pairs


def test_ras_bytes_one_subdomain_is_the_global_sweep():
    g = bench.algorithmic_bytes(12, 7, 5)
    r = bench.ras_algorithmic_bytes(12, 7, 5, (1, 1, 1), 1)
    assert r["cells"] == 12 * 7 * 5
    assert r["ilu_fwd"] == g["ilu_fwd"] and r["ilu_bwd"] == g["ilu_bwd"]


def test_ras_bytes_no_overlap_drops_the_cut_couplings():
    # 2 x 1 x 1 boxes of 6 x 7 x 5 without overlap: the 7 * 5 x-couplings across the cut are gone
    g = bench.algorithmic_bytes(12, 7, 5)
    r = bench.ras_algorithmic_bytes(12, 7, 5, (2, 1, 1), 0)
    assert r["cells"] == 12 * 7 * 5
    assert r["ilu_fwd"] == g["ilu_fwd"] - 72 * 7 * 5


def test_ras_bytes_match_brute_force():
    for dims, parts, ov in [((9, 7, 5), (3, 2, 1), 1), ((8, 8, 6), (2, 2, 2), 2), ((10, 3, 4), (3, 1, 2), 1)]:
        c, nl = brute_ras(*dims, parts, ov)
        r = bench.ras_algorithmic_bytes(*dims, parts, ov)
        assert (r["cells"], r["pairs"]) == (c, nl)
        assert r["ilu_fwd"] == 72 * nl + 48 * c and r["ilu_bwd"] == 72 * (nl + c) + 48 * c


def test_global_bytes_closed_form():
    nx, ny, nz = 6, 5, 4
    b = bench.algorithmic_bytes(nx, ny, nz)
    c = nx * ny * nz
    nl = (nx - 1) * ny * nz + nx * (ny - 1) * nz + nx * ny * (nz - 1)
    assert b["nnzb"] == 2 * nl + c
    assert b["spmv"] == 72 * (2 * nl + c) + 24 * 3 * c
