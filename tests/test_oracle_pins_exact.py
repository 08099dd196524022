"""More pins of the CPU oracle, each against a fact that does not come from
its code: an independent per-voxel evaluation of the membership rule, the
printed Eq. (1) in the planar case where it is exact, the rounding mode of
the fixed-point grid at exact half steps, the order of front-to-back
compositing with two different colours, and the alpha-layer limit of culling
rays at M - 1 and M blockers (arXiv 2510.09081, Sections 3.1, 3.2, 3.5).
"""
import math
from fractions import Fraction

import numpy as np
import pytest

from paper_2510_09081_amd import synth

from .test_oracle_pins import adversarial_segments, centre_camera, make_lineset, trace_centre

Q = 256


# ---------------------------------------------------------------------------
# Membership, evaluated voxel by voxel (Sec. 3.1, Alg. 1 with the projected
# radius that is conservative in 3D).  The oracle enumerates slab boxes with
# floor divisions; here every voxel of the capsule's box is tested on its own
# with integer inequalities, so a box one voxel too wide or narrow, a slab
# interval taken at the wrong ends, or a half-width built from the wrong
# direction component shows up as a set difference.


def ceil_isqrt(n):
    """Smallest w >= 0 with w * w >= n (exact, Python integers)."""
    if n <= 0:
        return 0
    w = math.isqrt(n)
    return w if w * w == n else w + 1


def voxel_in_set(A, B, rq, G, v):
    """Is voxel v in the capsule's voxel set?  One voxel, no enumeration."""
    d = [B[c] - A[c] for c in range(3)]
    a0 = 0
    for c in (1, 2):
        if abs(d[c]) > abs(d[a0]):
            a0 = c
    if d[a0] < 0:
        A, B = B, A
        d = [-x for x in d]
    D = d[a0]
    lo = [min(A[c], B[c]) - rq for c in range(3)]
    hi = [max(A[c], B[c]) + rq for c in range(3)]
    for c in range(3):
        # the closed cube of v touches the closed capsule box, inside the grid
        if not (0 <= v[c] < G[c] and v[c] * Q <= hi[c] and (v[c] + 1) * Q >= lo[c]):
            return False
    if D == 0:
        return True  # a ball: its box
    x = v[a0]
    ta, tb = max(lo[a0], x * Q), min(hi[a0], (x + 1) * Q)
    for i in range(3):
        if i == a0:
            continue
        ca = A[i] * D + d[i] * (ta - A[a0])  # the line's coordinate i at ta, scaled by D
        cb = A[i] * D + d[i] * (tb - A[a0])
        W = ceil_isqrt(rq * rq * (D * D + d[i] * d[i]))  # r sqrt(1 + (d_i/D)^2), scaled by D, rounded up
        if not (v[i] * Q * D <= max(ca, cb) + W and (v[i] + 1) * Q * D >= min(ca, cb) - W):
            return False
    return True


def per_voxel_set(A, B, rq, G):
    rng = [range(max(0, (min(A[c], B[c]) - rq - 1) // Q), min(G[c] - 1, (max(A[c], B[c]) + rq) // Q) + 1)
           for c in range(3)]
    return {(x, y, z) for x in rng[0] for y in rng[1] for z in rng[2] if voxel_in_set(A, B, rq, G, (x, y, z))}


def test_membership_equals_per_voxel_evaluation(orc):
    """>= 10^4 random and adversarial segments at several radii, lengths up
    to 6 voxels, on a non-cubic grid they partly leave."""
    G = (24, 20, 16)
    rng = np.random.default_rng(2510)
    segs = []
    for rq in (0, 51, 90, 128, 200, 333):
        for A, B in adversarial_segments(rng, 16, 0):
            segs.append((A, B, rq))
    while len(segs) < 10_500:
        A = rng.integers(-2 * Q, np.array(G) * Q + 2 * Q)
        L = rng.uniform(0, 6) * Q
        dv = rng.normal(size=3)
        if rng.random() < 0.3:  # exact ties between the largest components, and zero minors
            dv = np.array([1.0, rng.choice([1.0, -1.0]), rng.choice([0.0, 1.0, -1.0])])[rng.permutation(3)]
        dv = dv / np.linalg.norm(dv) * L
        B = np.rint(A + dv).astype(int)
        rq = int(rng.choice([0, 1, 51, 90, 128, 127, 129, 255, 256, 300]))
        segs.append((tuple(int(a) for a in A), tuple(int(b) for b in B), rq))
    n_nonempty = 0
    for A, B, rq in segs:
        got = orc.segment_voxels(A, B, rq, G)
        gset = {tuple(int(c) for c in v) for v in got}
        assert len(gset) == len(got), (A, B, rq)  # each voxel once
        exp = per_voxel_set(A, B, rq, G)
        assert gset == exp, (A, B, rq, sorted(gset ^ exp)[:6])
        n_nonempty += bool(exp)
    assert n_nonempty > 7000


# Pythagorean directions make |d| and the printed radius rational, so Eq. (1)
# can be evaluated exactly.  With one minor component zero (the planar case of
# the paper's traversal figure) the printed radius r / sqrt(1 - (d_i/|d|)^2)
# equals the conservative one, and the oracle's slab boxes must be the boxes
# the printed radius gives: the same set.
PLANAR = [  # (D, d_i) in whole voxels; D > |d_i|, D^2 + d_i^2 a square
    (4, 3), (4, -3), (12, 5), (12, -5), (15, 8), (24, 7), (8, 6), (3, 0)]


def eq1_planar_set(A, B, rq, G, i_minor):
    """Voxel set with the slab boxes of Alg. 1 and the printed Eq. (1) radius,
    in exact rationals (the slab ends are those of the oracle's reading: the
    capsule box, closed at both ends)."""
    d = [B[c] - A[c] for c in range(3)]
    a0 = max(range(3), key=lambda c: (abs(d[c]), -c))
    if d[a0] < 0:
        A, B = B, A
        d = [-x for x in d]
    D = d[a0]
    norm = Fraction(math.isqrt(sum(x * x for x in d)))
    assert norm * norm == sum(x * x for x in d)
    r = Fraction(rq, Q)
    lo = [min(A[c], B[c]) - rq for c in range(3)]
    hi = [max(A[c], B[c]) + rq for c in range(3)]
    box = [range(max(0, (lo[c] - 1) // Q), min(G[c] - 1, hi[c] // Q) + 1) for c in range(3)]
    out = set()
    for x in box[a0]:
        ta = Fraction(max(lo[a0], x * Q), Q)
        tb = Fraction(min(hi[a0], (x + 1) * Q), Q)
        ranges = {}
        for i in range(3):
            if i == a0:
                continue
            rhat = r / Fraction(math.isqrt(((norm * norm - d[i] * d[i]) / (norm * norm)).numerator),
                                math.isqrt(((norm * norm - d[i] * d[i]) / (norm * norm)).denominator))
            p0 = Fraction(A[i], Q) + Fraction(d[i], D) * (ta - Fraction(A[a0], Q))
            p1 = Fraction(A[i], Q) + Fraction(d[i], D) * (tb - Fraction(A[a0], Q))
            jlo, jhi = min(p0, p1) - rhat, max(p0, p1) + rhat
            # voxels whose closed interval [j, j + 1] touches [jlo, jhi]
            ranges[i] = [j for j in box[i] if j <= jhi and j + 1 >= jlo]
        others = [c for c in range(3) if c != a0]
        for j in ranges[others[0]]:
            for k in ranges[others[1]]:
                v = [0, 0, 0]
                v[a0], v[others[0]], v[others[1]] = x, j, k
                out.add(tuple(v))
    return out


@pytest.mark.parametrize("Dv,dv", PLANAR)
@pytest.mark.parametrize("rq", [128, 90, 256])
def test_membership_planar_case_is_equation1(orc, Dv, dv, rq):
    G = (40, 40, 40)
    rng = np.random.default_rng(Dv * 100 + dv + rq)
    for trial in range(12):
        axes = rng.permutation(3)  # major, minor with d_i, minor with zero
        A = [int(a) for a in rng.integers(8 * Q, 16 * Q, size=3)]
        s = int(rng.choice([32, 64, 256, 128 + 64]))  # step scale in Q units (lengths 0.5..1 of the triple)
        d = [0, 0, 0]
        d[axes[0]] = Dv * s * (1 if trial % 2 == 0 else -1)
        d[axes[1]] = dv * s
        B = [A[c] + d[c] for c in range(3)]
        got = {tuple(int(c) for c in v) for v in orc.segment_voxels(A, B, rq, G)}
        exp = eq1_planar_set(A, B, rq, G, axes[1])
        assert got == exp, (A, B, rq, sorted(got ^ exp)[:6])


# ---------------------------------------------------------------------------
# Quantization rounding (fixed-point grid, 1/256 voxel): round to nearest, ties
# to even, at inputs that are not on the grid.


def quant_lineset(xs, vs, origin):
    xyz = np.zeros((len(xs), 3), np.float32)
    xyz[:, 0] = xs
    xyz[:, 1] = origin[1] + np.float32(3.0) * vs  # on the grid
    xyz[:, 2] = origin[2] + np.float32(5.0) * vs
    return synth.LineSet(xyz=xyz, offsets=np.array([0, len(xs)], np.int32), radius=float(vs) * 0.5,
                         origin=np.asarray(origin, np.float32), voxel_size=float(vs), dims=(64, 64, 64))


@pytest.mark.parametrize("origin_x", [0.0, 0.25, -0.5])
def test_quantization_round_to_nearest_even(orc, origin_x):
    """With voxel size 2^-6 the scale is 2^14, so x = o + (q + 1/2) 2^-14 is
    a binary32 number whose scaled offset is exactly q + 1/2: the grid value
    must be the even neighbour.  One ulp above and below must round up and
    down.  Truncation, floor, or ties away from zero each fail some case."""
    vs = np.float32(2.0 ** -6)
    origin = np.array([origin_x, 0.0, 0.0], np.float32)
    qs = [0, 1, 2, 3, 10, 11, 1001, 1002, 4095, -1, -2, -7, -8, -1000, -1001]
    xs, exp = [], []
    for q in qs:
        half = np.float32(origin_x + (q + 0.5) * 2.0 ** -14)
        assert float(half) == origin_x + (q + 0.5) * 2.0 ** -14  # exactly representable
        even = q if q % 2 == 0 else q + 1
        xs += [half, np.nextafter(half, np.float32(np.inf)), np.nextafter(half, np.float32(-np.inf))]
        exp += [even, q + 1, q]
        off = np.float32(origin_x + q * 2.0 ** -14 + 0.3 * 2.0 ** -14)  # not a half step: nearest
        xs.append(off)
        exp.append(int(round((float(off) - origin_x) * 2.0 ** 14)))
    ing = orc.ingest(quant_lineset(np.array(xs, np.float32), vs, origin))
    assert ing.status == 0
    assert ing.q[:, 0].tolist() == exp
    assert ing.q[:, 1].tolist() == [3 * Q] * len(xs) and ing.q[:, 2].tolist() == [5 * Q] * len(xs)


def test_quantization_radius_and_eye_round_half_even(orc):
    """The radius and the eye are quantized in binary64 with ties to even:
    r = 0.5/256 voxel -> 0 (even), 1.5/256 -> 2, 2.5/256 -> 2."""
    vs = 2.0 ** -6
    for r_steps, exp in ((0.5, 0), (1.5, 2), (2.5, 2), (127.5, 128), (128.5, 128), (0.49, 0), (0.51, 1)):
        ls = quant_lineset(np.array([0.1, 0.2], np.float32), np.float32(vs), np.zeros(3, np.float32))
        ls = synth.LineSet(xyz=ls.xyz, offsets=ls.offsets, radius=float(np.float32(r_steps * vs / Q)),
                           origin=ls.origin, voxel_size=ls.voxel_size, dims=ls.dims)
        assert orc.ingest(ls).rq == exp, r_steps
    ls = quant_lineset(np.array([0.1, 0.2], np.float32), np.float32(vs), np.zeros(3, np.float32))
    eye = np.array([(7 + 0.5) * vs / Q, (8 + 0.5) * vs / Q, -(3 + 0.5) * vs / Q], np.float32)
    assert orc.eye_q(eye, ls).tolist() == [8, 8, -4]


# ---------------------------------------------------------------------------
# Compositing order (Sec. 3.5: front to back, in visibility order)


@pytest.mark.parametrize("alpha", [0.3, 0.5, 0.8])
def test_trace_two_colours_composite_front_to_back(orc, alpha):
    """A red line (along x) in front of a green line (along y), seen from
    above: C = alpha red + alpha (1 - alpha) green, A = 1 - (1 - alpha)^2.
    Back-to-front order would swap the two weights."""
    G = 64
    front = [[20 + k, 32.3, 40.5] for k in range(25)]   # along x: colour (1, 0, 0)
    back = [[32.4, 20 + k, 20.5] for k in range(25)]    # along y: colour (0, 1, 0)
    ls = make_lineset([back, front], G, 0.5)           # the back line has the lower ids
    cam = centre_camera((32.4, 32.3, 60), (32.4, 32.3, 0), G)
    tr, _ = trace_centre(orc, ls, cam, mode=1, alpha=alpha)
    assert tr.n_comp[0] == 2
    exp = [alpha, alpha * (1 - alpha), 0.0, 1 - (1 - alpha) ** 2]
    assert np.allclose(tr.rgba[0], exp, rtol=0, atol=1e-12), (tr.rgba[0], exp)
    assert tr.id[0] >= 25  # the first hit is the front (red) line
    trb, _ = trace_centre(orc, ls, cam, mode=0)
    assert np.allclose(trb.rgba[0], [1, 0, 0, 1], rtol=0, atol=1e-12)


# ---------------------------------------------------------------------------
# Alpha-layer culling (Sec. 3.2 culling rays; the layer limit M(alpha))


@pytest.mark.parametrize("alpha,M", [(0.2, 25), (0.3, 16), (0.5, 9)])
def test_alpha_culling_hides_behind_M_blockers_only(orc, alpha, M):
    """An occupied voxel under a column of k blocking voxels, the eye straight
    above: visible for k = M - 1, hidden for k = M (alpha culling), hidden
    for k = 1 (opaque culling), visible for any k without culling."""
    lim = orc.cull_limit(orc.CULL_ALPHA, alpha)
    assert lim == M
    G = (8, 8, 40)
    v = (3, 5, 1)
    eyeq = np.array([3 * Q + 128, 5 * Q + 128, 60 * Q + 7], np.int64)
    for k, visible in ((M - 1, True), (M, False), (M + 3, False), (0, True)):
        words = np.zeros(G[::-1], np.uint32)
        words[v[2], v[1], v[0]] = 1
        blk = np.zeros(G[::-1], np.uint8)
        blk[v[2] + 1:v[2] + 1 + k, v[1], v[0]] = 1
        vis = orc.visibility(words, blk, eyeq, lim)
        assert bool(vis[v[2], v[1], v[0]]) == visible, (k, M)
        n, _ = orc.culling_ray(v, eyeq, blk, 10 ** 6)
        assert n == k
        if k >= 1:
            assert orc.visibility(words, blk, eyeq, orc.cull_limit(orc.CULL_OPAQUE))[v[2], v[1], v[0]] == 0
        assert orc.visibility(words, blk, eyeq, orc.cull_limit(orc.CULL_NONE))[v[2], v[1], v[0]] == 1
    # blockers beside the column do not count: the ray meets only the column's interiors
    words = np.zeros(G[::-1], np.uint8).astype(np.uint32)
    words[v[2], v[1], v[0]] = 1
    blk = np.ones(G[::-1], np.uint8)
    blk[:, v[1], v[0]] = 0
    assert orc.visibility(words, blk, eyeq, 1)[v[2], v[1], v[0]] == 1


def test_alpha_culling_through_a_wall_of_lines(orc):
    """The same through the whole build: under a thick wall of lines the
    voxels behind it are culled with alpha = 0.5 (M = 9) only where the ray
    meets at least 9 blocking voxels, which is where the wall is at least 11
    voxels thick (erosion removes one layer on each face)."""
    G = 32
    polys = []
    for z in range(4, 19):          # a wall 15 voxels thick in z under x < 16 ...
        for y in range(2, 30):
            polys.append([[2, y + 0.5, z + 0.5], [15.5, y + 0.5, z + 0.5]])
    for z in range(4, 10):          # ... and 6 voxels thick under x >= 16
        for y in range(2, 30):
            polys.append([[16.5, y + 0.5, z + 0.5], [30, y + 0.5, z + 0.5]])
    polys.append([[4, 16.5, 1.5], [28, 16.5, 1.5]])  # the line under the wall
    ls = make_lineset(polys, G, 0.75)
    eye = np.array([16.0, 16.5, 200.0], np.float32) / G  # far above: near-vertical rays
    fr = orc.build_frame(ls, eye, orc.CULL_ALPHA, alpha=0.5)
    assert fr.limit == 9
    row = fr.vis[1, 16, :]
    assert row[5:13].sum() == 0            # under the thick part: hidden
    assert row[19:27].all()                # under the thin part: visible
    fo = orc.build_frame(ls, eye, orc.CULL_OPAQUE)
    assert fo.vis[1, 16, 19:27].sum() == 0  # opaque culling hides both


# ---------------------------------------------------------------------------
# Segments and clip planes (Sec. 3.1: capsules clipped at interior joints by
# the plane whose normal is the polyline's tangent there; Sec. 3.3: primitive
# i is the segment from vertex i to vertex i + 1 of one polyline).


def test_segment_flags_and_clip_normals_from_the_polyline_definition(orc):
    """Ragged polylines (one vertex, two, many; a repeated vertex giving a zero tangent): vertex i starts a
    segment iff vertex i + 1 belongs to the same polyline, and only vertices with a neighbour on both sides
    and a non-zero central difference carry a clip normal, which is that difference normalized (checked in
    binary64 against the integer positions, to the binary32 rounding of the normalization)."""
    polys = [[[2.0, 2.0, 2.0]],
             [[3.0, 3.0, 3.0], [5.0, 7.0, 4.0]],
             [[1.0, 1.0, 1.0], [4.0, 2.0, 1.0], [6.5, 3.25, 2.0], [6.5, 6.0, 5.5], [2.0, 9.0, 8.0]],
             [[8.0, 8.0, 8.0], [9.0, 8.0, 8.0], [8.0, 8.0, 8.0], [8.0, 8.0, 8.0]]]
    ls = make_lineset(polys, 16, 0.5)
    ing = orc.ingest(ls)
    off = ls.offsets
    q = ing.q.astype(np.int64)
    for p in range(len(off) - 1):
        for i in range(off[p], off[p + 1]):
            assert ing.seg_valid[i] == (i + 1 < off[p + 1]), i
            inner = off[p] < i < off[p + 1] - 1
            T = (q[i + 1] - q[i - 1]) if inner else np.zeros(3, np.int64)
            if inner and (T != 0).any():
                assert ing.interior[i] == 1, i
                n = T / math.sqrt(float((T * T).sum()))
                assert np.abs(ing.nrm[i].astype(np.float64) - n).max() < 2e-7, i
            else:
                assert ing.interior[i] == 0 and (ing.nrm[i] == 0).all(), i
    # (9, 8, 8) sits between two copies of (8, 8, 8): zero tangent, no clip; the next vertex has one
    assert ing.interior[off[3] + 2] == 1 and ing.interior[off[3] + 1] == 0


# ---------------------------------------------------------------------------
# The comparison voxelizers of Sec. 4.1 (Table 2): a thin line walk ("DDA")
# and the capsule's bounding box.  Pinned against their definitions evaluated
# here with Python fractions, and against the capsule voxelizer they are
# compared with.


def _thin_reference(A, B, G):
    """Voxels whose open interior the open segment (A, B) meets, plus the cells of A and B (Q units)."""
    out = set()
    ca = tuple(a // Q for a in A)
    cb = tuple(b // Q for b in B)
    for v in (ca, cb):
        if all(0 <= v[c] < G for c in range(3)):
            out.add(v)
    lo_v = [max(min(ca[c], cb[c]) - 1, 0) for c in range(3)]
    hi_v = [min(max(ca[c], cb[c]) + 1, G - 1) for c in range(3)]
    for x in range(lo_v[0], hi_v[0] + 1):
        for y in range(lo_v[1], hi_v[1] + 1):
            for z in range(lo_v[2], hi_v[2] + 1):
                t0, t1 = Fraction(0), Fraction(1)
                ok = True
                for c, vc in enumerate((x, y, z)):
                    d = B[c] - A[c]
                    lo, hi = vc * Q, (vc + 1) * Q
                    if d == 0:
                        ok &= lo < A[c] < hi
                        continue
                    ta, tb = Fraction(lo - A[c], d), Fraction(hi - A[c], d)
                    t0, t1 = max(t0, min(ta, tb)), min(t1, max(ta, tb))
                if ok and t0 < t1:
                    out.add((x, y, z))
    return out


def _set(arr):
    return {tuple(int(c) for c in v) for v in arr}


def test_thin_line_voxels_equal_their_definition(orc):
    rng = np.random.default_rng(41)
    G = 12
    segs = [((Q * 2 + 128, Q * 2 + 128, Q * 2 + 128), (Q * 9 + 128, Q * 2 + 128, Q * 2 + 128)),  # axis-aligned
            ((Q * 1, Q * 1, Q * 1), (Q * 5, Q * 5, Q * 5)),          # through voxel corners
            ((Q * 3, Q * 4 + 128, Q * 5 + 128), (Q * 8, Q * 4 + 128, Q * 5 + 128)),  # starts on a face
            ((Q * 4, Q * 4, Q * 6 + 77), (Q * 7, Q * 7, Q * 6 + 77)),  # along a face diagonal, edge ties
            ((Q * 3, Q * 5, Q * 2), (Q * 9, Q * 5, Q * 2)),          # lies on voxel faces: no interior is met
            ((Q * 6 + 5, Q * 6 + 9, Q * 6 + 11), (Q * 6 + 5, Q * 6 + 9, Q * 6 + 11)),  # zero length
            ((-Q * 2, Q * 3 + 7, Q * 4 + 1), (Q * 14, Q * 5 + 3, Q * 6 + 200))]  # leaves the grid
    for _ in range(300):
        A = rng.integers(-Q, (G + 1) * Q, 3)
        B = A + rng.integers(-4 * Q, 4 * Q, 3)
        if rng.uniform() < 0.3:  # snap some coordinates to voxel faces
            A = np.where(rng.uniform(size=3) < 0.5, (A // Q) * Q, A)
            B = np.where(rng.uniform(size=3) < 0.5, (B // Q) * Q, B)
        segs.append((tuple(int(a) for a in A), tuple(int(b) for b in B)))
    for A, B in segs:
        got = _set(orc.segment_voxels(A, B, 0, (G, G, G), mode=orc.VOX_THIN))
        assert got == _thin_reference(A, B, G), (A, B)
    # closed forms: a straight run of voxels; the corner diagonal visits only the diagonal voxels
    assert _set(orc.segment_voxels(*segs[0], 0, (G, G, G), mode=orc.VOX_THIN)) == {(x, 2, 2) for x in range(2, 10)}
    assert _set(orc.segment_voxels(*segs[1], 0, (G, G, G), mode=orc.VOX_THIN)) == {(k, k, k) for k in range(1, 6)}
    assert _set(orc.segment_voxels(*segs[4], 0, (G, G, G), mode=orc.VOX_THIN)) == {(3, 5, 2), (9, 5, 2)}


def test_comparison_voxelizers_bracket_the_capsule(orc):
    """thin line (radius ignored) <= capsule voxels <= capsule AABB voxels, and the AABB set is exactly the
    voxels whose closed cube meets the capsule's closed bounding box."""
    rng = np.random.default_rng(43)
    G = 12
    for _ in range(300):
        A = rng.integers(0, G * Q, 3)
        B = A + rng.integers(-5 * Q, 5 * Q, 3)
        rq = int(rng.choice([0, 51, 128, 200]))
        thin = _set(orc.segment_voxels(A, B, rq, (G, G, G), mode=orc.VOX_THIN))
        caps = _set(orc.segment_voxels(A, B, rq, (G, G, G)))
        box = _set(orc.segment_voxels(A, B, rq, (G, G, G), mode=orc.VOX_AABB))
        assert thin <= caps <= box, (A, B, rq)
        lo = np.minimum(A, B) - rq
        hi = np.maximum(A, B) + rq
        ref = {(x, y, z) for x in range(G) for y in range(G) for z in range(G)
               if all(v * Q <= h and l <= (v + 1) * Q for v, l, h in zip((x, y, z), lo, hi))}
        assert box == ref, (A, B, rq)


# ---------------------------------------------------------------------------
# Per-segment colour and opacity (the boundary's optional RGBA per segment):
# each hit is composited with its own opacity, front to back.


def test_trace_per_segment_rgba_composite(orc):
    """Front line (colour c1, opacity a1) over a back line (c2, a2), seen from above:
    C = a1 c1 + (1 - a1) a2 c2, A = 1 - (1 - a1)(1 - a2); opaque shows c1 with alpha 1."""
    G = 64
    front = [[20 + k, 32.3, 40.5] for k in range(25)]
    back = [[32.4, 20 + k, 20.5] for k in range(25)]
    ls = make_lineset([back, front], G, 0.5)
    cam = centre_camera((32.4, 32.3, 60), (32.4, 32.3, 0), G)
    c1, a1, c2, a2 = np.array([0.2, 0.7, 0.1]), 0.6, np.array([0.9, 0.3, 0.5]), 0.25
    rgba = np.zeros((ls.n_vertices, 4), np.float32)
    rgba[:25] = np.append(c2, a2)     # back line: vertices 0..24
    rgba[25:] = np.append(c1, a1)     # front line: vertices 25..49
    fr = orc.build_frame(ls, cam.eye, 0)
    pix = [(cam.height // 2) * cam.width + cam.width // 2]
    tr = orc.trace(fr, ls, cam, pix, 1, alpha=0.9, seg_rgba=rgba)
    f32 = lambda v: np.float32(v).astype(np.float64)  # noqa: E731 - the colours are stored in binary32
    A1, A2 = f32(a1), f32(a2)
    exp_c = A1 * f32(c1) + (1 - A1) * A2 * f32(c2)
    assert tr.n_comp[0] == 2
    assert np.allclose(tr.rgba[0][:3], exp_c, rtol=0, atol=1e-12)
    assert abs(tr.rgba[0][3] - (1 - (1 - A1) * (1 - A2))) < 1e-12
    tro = orc.trace(fr, ls, cam, pix, 0, seg_rgba=rgba)
    assert np.allclose(tro.rgba[0], np.append(f32(c1), 1.0), rtol=0, atol=1e-12)


def test_trace_rgba_equal_to_the_default_reproduces_it(orc):
    """RGBA rows holding |unit tangent| and the default opacity give the default image (the two colour sources
    agree), on a random-walk set, opaque and transparent."""
    ls = synth.random_walk_set(seed=13, n_poly=30, n_seg=20, G=32)
    cam = synth.grid_camera(ls, 48, 36)
    fr = orc.build_frame(ls, cam.eye, 0)
    q = fr.ing.q.astype(np.float64)
    d = np.zeros_like(q)
    d[:-1] = q[1:] - q[:-1]
    n = np.linalg.norm(d, axis=1, keepdims=True)
    col = np.where(n > 0, np.abs(d) / np.where(n > 0, n, 1), 0.0)
    pix = np.arange(cam.width * cam.height)
    for mode, alpha in ((0, 1.0), (1, 0.5)):  # 0.5 and the colours' binary32 rounding: compare loosely
        rgba = np.concatenate([col, np.full((len(q), 1), alpha)], axis=1).astype(np.float32)
        a = orc.trace(fr, ls, cam, pix, mode, alpha=alpha)
        b = orc.trace(fr, ls, cam, pix, mode, alpha=alpha, seg_rgba=rgba)
        assert np.array_equal(a.id, b.id)
        assert np.abs(a.rgba - b.rgba).max() < 1e-6
        assert (a.id >= 0).sum() > 100


# ---------------------------------------------------------------------------
# Voxel-space shading (Sec. 3.4): cone-traced ambient occlusion over the
# occupancy pyramid, a directional shadow ray, visible voxels only.  Pinned
# with synthetic pyramids whose answers are closed forms.


def _pyramid(G, fill):
    """Dense occupancy levels (uint16, 1/256 units) of a G^3 grid, every level filled by fill(level, dims)."""
    lv, d = [], (G, G, G)
    while True:
        lv.append(fill(len(lv), d))
        if d == (1, 1, 1):
            return lv
        d = tuple((x + 1) // 2 for x in d)


def test_shade_cone_directions_fibonacci(orc):
    K = 16
    U = orc.shade_dirs(K).astype(np.float64)
    golden = math.pi * (3 - math.sqrt(5))
    for k in range(K):
        z = 1 - (2 * k + 1) / K
        assert U[k, 2] == round(256 * z)  # evenly spaced heights (none is a half-step here)
        assert abs(np.linalg.norm(U[k]) / 256 - 1) < 2e-3
        phi = math.atan2(U[k, 1], U[k, 0])
        assert abs(math.remainder(phi - golden * k, 2 * math.pi)) < 0.02 or abs(z) > 0.99


def test_shade_constant_field_closed_form(orc):
    """Every level holds occupancy 1/4: a voxel whose samples all stay inside the grid has AO = (3/4)^J; the
    shadow ray along +z crosses G - 1 - z voxels, S = (3/4)^(G-1-z); lit = AO (a + (1 - a) S)."""
    G, J, amb = 64, 4, 0.3
    occ = _pyramid(G, lambda L, d: np.full(d[::-1], 64, np.uint16))
    vis = np.zeros((G, G, G), np.uint8)
    pts = [(32, 32, 32), (30, 35, 40), (20, 25, 44)]
    for x, y, z in pts:
        vis[z, y, x] = 1
    ao, sh, lit = orc.shade(occ, vis, n_cones=16, n_samples=J, light=(0, 0, 1), ambient=amb)
    for x, y, z in pts:
        assert ao[z, y, x] == 0.75 ** J
        assert sh[z, y, x] == 0.75 ** (G - 1 - z)
        assert abs(lit[z, y, x] - 0.75 ** J * (amb + (1 - amb) * 0.75 ** (G - 1 - z))) < 1e-15
    assert (lit[vis == 0] == 0).all()


def test_shade_empty_surroundings_and_walk_ties(orc):
    """With nothing around, AO = S = lit = 1.  A diagonal light in the xy plane from a voxel centre passes the
    corner line shared with its x and y neighbours: a full voxel there casts no shadow (tied axes step
    together), a full voxel on the diagonal casts a full one, a half-full one halves the light."""
    G = 32
    zero = _pyramid(G, lambda L, d: np.zeros(d[::-1], np.uint16))
    vis = np.zeros((G, G, G), np.uint8)
    vis[10, 10, 10] = 1
    ao, sh, lit = orc.shade(zero, vis, light=(1, 1, 0))
    assert ao[10, 10, 10] == 1 and sh[10, 10, 10] == 1 and lit[10, 10, 10] == 1
    for cells, expect in (([(11, 10, 10), (10, 11, 10)], 1.0), ([(12, 12, 10)], 0.0), ([(13, 13, 10)], 0.5)):
        lv = [z.copy() for z in zero]
        for (x, y, z) in cells:
            lv[0][z, y, x] = 128 if expect == 0.5 else 256
        _, sh, _ = orc.shade(lv, vis, light=(1, 1, 0))
        assert sh[10, 10, 10] == expect, (cells, sh[10, 10, 10])


def test_trace_shaded_colour_is_the_hit_voxels_value(orc):
    """Shading scales each hit's colour by the value of the voxel holding the hit point: with a shading
    field that is constant per x-slab, the opaque colour of a hit equals |tangent| times the value of the
    slab its depth lands in, and a constant field s scales a transparent composite by exactly s."""
    ls = synth.random_walk_set(seed=13, n_poly=30, n_seg=20, G=32)
    cam = synth.grid_camera(ls, 48, 36)
    fr = orc.build_frame(ls, cam.eye, 0)
    pix = np.arange(cam.width * cam.height)
    base0 = orc.trace(fr, ls, cam, pix, 0)
    base1 = orc.trace(fr, ls, cam, pix, 1, alpha=0.4)
    slab = np.broadcast_to(np.linspace(0.2, 1.0, 32)[None, None, :], fr.vis.shape).copy()
    sh0 = orc.trace(fr, ls, cam, pix, 0, lit=slab)
    assert np.array_equal(sh0.id, base0.id)
    hit = base0.id >= 0
    eye = orc.eye_q(cam.eye, ls) / 256.0
    dirs = orc.ray_dirs(cam, pix).astype(np.float64)
    P = eye + dirs[hit] * base0.t[hit][:, None]
    s = np.linspace(0.2, 1.0, 32)[np.floor(P[:, 0]).astype(int)]
    ok = (np.abs(P[:, 0] - np.round(P[:, 0])) > 1e-6)  # hit points not on an x face
    assert np.allclose(sh0.rgba[hit][ok, :3], base0.rgba[hit][ok, :3] * s[ok][:, None], atol=1e-12)
    const = np.full(fr.vis.shape, 0.625)
    sh1 = orc.trace(fr, ls, cam, pix, 1, alpha=0.4, lit=const)
    assert np.allclose(sh1.rgba[:, :3], 0.625 * base1.rgba[:, :3], atol=1e-12)
    assert np.allclose(sh1.rgba[:, 3], base1.rgba[:, 3], atol=1e-12)
