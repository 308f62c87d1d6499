"""Set-up of the micro/mesopore study (Section 5.3), on the CPU: the three
variants share their ionomer and differ only by pores carved inside carbon that
was there in the original, away from every carbon-ionomer face."""
import numpy as np

from paper_1410_1914_amd import pore_study as ps

PORE, CARBON, PT, IONOMER = 0, 1, 2, 3


def _six_neighbours(mask):
    out = np.zeros_like(mask)
    for ax in (0, 1):
        out |= np.roll(mask, 1, ax) | np.roll(mask, -1, ax)
    out[:, :, 1:] |= mask[:, :, :-1]
    out[:, :, :-1] |= mask[:, :, 1:]
    return out


def test_variants_differ_only_by_pores_carved_in_carbon():
    n = 40
    base = ps.structure("original", 3, n)
    assert abs((base == CARBON).mean() - 0.55) < 0.01 and abs((base == IONOMER).mean() - 0.15) < 0.01
    for name in ("A1", "A2"):
        ph = ps.structure(name, 3, n)
        carved = (ph == PORE) & (base != PORE)
        assert np.array_equal(ph == IONOMER, base == IONOMER), name
        assert (base[carved] == CARBON).all(), name               # carved only out of carbon
        assert np.array_equal(ph[~carved], base[~carved]), name    # nothing else changed
        assert abs(carved.mean() - 0.10) < 0.01, name
        assert not (carved & _six_neighbours(base == IONOMER)).any(), name  # ionomer contact kept
