"""Pins from values the paper prints: the star2d4r example kernel of Sec. 5.

tests/golden/star2d4r_listing_weights.txt holds the listing's 17 weights as
printed.  They pin the encoding the GPU suite tests use
(synth.listing_star2d4r_weights), and, through closed forms computed from
the fixture's own moments, the oracle's general 2D stencil: on a quadratic
field a symmetric stencil returns
    m0 * u + (b_xx * M2x + b_yy * M2y),
    m0 = sum w,  M2x = sum w dx^2,  M2y = sum w dy^2,
for u = a + b_x x + b_y y + b_xx x^2 + b_yy y^2 away from the zero frame.
The listing's x and y weights differ (M2x != M2y), so a transposed axis, a
dropped term or a wrong sign fails.
"""

import os

import numpy as np

import oracle
import synth

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "star2d4r_listing_weights.txt")


def load_golden():
    terms = []
    for line in open(GOLDEN):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        dx, dy, w = line.split()
        terms.append((int(dx), int(dy), float(w)))
    return terms


def test_fixture_is_the_listing_shape():
    terms = load_golden()
    assert len(terms) == 17
    offs = {(dx, dy) for dx, dy, _ in terms}
    assert len(offs) == 17
    assert all(dx == 0 or dy == 0 for dx, dy in offs) and max(abs(dx) + abs(dy) for dx, dy in offs) == 4
    w = {(dx, dy): v for dx, dy, v in terms}
    assert all(w[(dx, dy)] == w[(-dx, -dy)] for dx, dy in offs)


def test_synth_encoding_matches_the_printed_weights():
    w = synth.listing_star2d4r_weights()
    expect = np.zeros((9, 9))
    for dx, dy, v in load_golden():
        expect[4 + dy, 4 + dx] = v
    assert np.array_equal(w, expect)


def test_oracle_general_stencil_on_quadratics():
    terms = load_golden()
    m0 = sum(v for _, _, v in terms)
    m2x = sum(v * dx * dx for dx, _, v in terms)
    m2y = sum(v * dy * dy for _, dy, v in terms)
    assert abs(m2x - m2y) > 1.0          # the listing's axes differ
    w = np.zeros((9, 9))
    for dx, dy, v in terms:
        w[4 + dy, 4 + dx] = v
    ny, nx = 23, 29
    y, x = np.meshgrid(np.arange(ny, dtype=np.float64), np.arange(nx, dtype=np.float64), indexing="ij")
    a, bx, by, bxx, byy = 1.5, 0.25, -0.75, 0.125, -0.0625
    u = a + bx * x + by * y + bxx * x * x + byy * y * y
    got = oracle.stencil_general(u, w, 2)
    expect = m0 * u + bxx * m2x + byy * m2y
    core = (slice(4, ny - 4), slice(4, nx - 4))
    assert np.allclose(got[core], expect[core], rtol=1e-13, atol=1e-12)
    # at the frame the zero halo replaces the missing terms: brute force there
    pad = np.zeros((ny + 8, nx + 8))
    pad[4:-4, 4:-4] = u
    for (j, i) in [(0, 0), (0, nx - 1), (ny - 1, 0), (3, 17), (ny - 2, 5)]:
        ref = sum(v * pad[4 + j + dy, 4 + i + dx] for dx, dy, v in terms)
        assert abs(got[j, i] - ref) <= 1e-12 * (1 + abs(ref))
