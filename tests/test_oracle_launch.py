"""Pins of the oracle's launch grid (Sec. II.B, eqs. (1)-(2), ray count with
eq. (4)) against facts fixed independently of the oracle: textbook
geodesic constructions, closed-form counts, the icosahedral symmetry group,
high-precision decimal trigonometry, and the paper's qualitative claim that
equiangular division is more uniform than equidistant division."""
import math
from decimal import Decimal, getcontext

import numpy as np
import pytest

PHI = (1 + 5 ** 0.5) / 2


def ico_vertex_set():
    raw = []
    for a in (1, -1):
        for b in (PHI, -PHI):
            raw += [(0, a, b), (a, b, 0), (b, 0, a)]
    v = np.array(raw, float)
    return v / np.linalg.norm(v, axis=1, keepdims=True)


def ico_rotations():
    """The 60 rotations of the icosahedral group, built from vertex frames."""
    V = ico_vertex_set()
    adj = [(i, j) for i in range(12) for j in range(12) if i != j and V[i] @ V[j] > 0]

    def frame(a, b):
        e1 = a
        e2 = b - (b @ a) * a
        e2 /= np.linalg.norm(e2)
        return np.stack([e1, e2, np.cross(e1, e2)], axis=1)

    F0 = frame(V[adj[0][0]], V[adj[0][1]])
    rots = []
    for i, j in adj:
        R = frame(V[i], V[j]) @ F0.T
        W = V @ R.T
        # must permute the vertex set
        d = np.abs(W[:, None, :] - V[None, :, :]).max(axis=2).min(axis=1)
        if d.max() < 1e-12 and np.linalg.det(R) > 0:
            rots.append(R)
    return rots


def nearest_angles(P):
    """Angle from each point to its nearest other point (radians)."""
    G = P @ P.T
    np.fill_diagonal(G, -2.0)
    c = np.clip(G.max(axis=1), -1.0, 1.0)
    # accurate small angles: use chord length
    return 2.0 * np.arcsin(np.sqrt(np.maximum(0.0, 2.0 - 2.0 * c)) / 2.0)


def equidistant_grid(V, faces, n):
    pts = []
    for f in faces:
        A, B, Cc = V[list(f)]
        for i in range(n + 1):
            for j in range(n + 1 - i):
                k = n - i - j
                pts.append((i * A + j * B + k * Cc) / n)
    P = np.array(pts)
    P /= np.linalg.norm(P, axis=1, keepdims=True)
    # dedupe shared edge points
    key = np.round(P, 12)
    _, idx = np.unique(key, axis=0, return_index=True)
    return P[np.sort(idx)]


def ico_faces(V):
    adj = V @ V.T > 0
    np.fill_diagonal(adj, False)
    return [(i, j, k) for i in range(12) for j in range(i + 1, 12) for k in range(j + 1, 12)
            if adj[i, j] and adj[j, k] and adj[i, k]]


def octa_faces():
    V = np.array([[1, 0, 0], [-1, 0, 0], [0, 1, 0], [0, -1, 0], [0, 0, 1], [0, 0, -1]], float)
    F = [(a, b, c) for a in (0, 1) for b in (2, 3) for c in (4, 5)]
    return V, F


def test_ray_count_closed_form(orc):
    # N = 10 n^2 + 2 (stated with eq. (4)); 4412 rays at n = 21 (Sec. IV)
    for n in range(1, 40):
        assert orc.num_rays(n) == 10 * n * n + 2
        d = orc.launch_dirs(n)
        assert d.shape == (10 * n * n + 2, 3)
    assert orc.num_rays(21) == 4412


@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 7, 20, 21])
def test_unit_and_distinct(orc, n):
    d = orc.launch_dirs(n)
    assert np.abs(np.linalg.norm(d, axis=1) - 1.0).max() <= 4e-16
    # all directions distinct: nearest neighbour well above rounding
    assert nearest_angles(d).min() > 0.5 * math.atan(2.0) / n


def test_n1_is_icosahedron(orc):
    d = orc.launch_dirs(1)
    V = ico_vertex_set()
    dist = np.abs(d[:, None, :] - V[None, :, :]).max(axis=2)
    assert dist.min(axis=1).max() < 1e-15 and dist.min(axis=0).max() < 1e-15


def test_n2_is_frequency2_geodesic(orc):
    # n = 2: 12 vertices + 30 normalized edge midpoints (geodesic sphere, 42 points)
    d = orc.launch_dirs(2)
    V = ico_vertex_set()
    adj = V @ V.T > 0
    mids = [(V[i] + V[j]) / np.linalg.norm(V[i] + V[j]) for i in range(12) for j in range(i + 1, 12)
            if adj[i, j]]
    ref = np.concatenate([V, np.array(mids)])
    assert len(ref) == 42
    dist = np.abs(d[:, None, :] - ref[None, :, :]).max(axis=2)
    assert dist.min(axis=1).max() < 1e-15 and dist.min(axis=0).max() < 1e-15


@pytest.mark.parametrize("n", [3, 7, 20])
def test_equal_angles_along_edges(orc, n):
    # eq. (1) on layer 0: consecutive edge points subtend theta_0 / n, theta_0 = atan 2
    d = orc.launch_dirs(n)
    V = d[:12]
    adj = V @ V.T > 0
    e = 0
    th0 = math.atan(2.0)
    assert abs(math.degrees(th0) - 63.4349) < 1e-4
    for i in range(12):
        for j in range(i + 1, 12):
            if not adj[i, j]:
                continue
            pts = np.concatenate([V[i:i + 1], d[12 + e * (n - 1): 12 + (e + 1) * (n - 1)], V[j:j + 1]])
            a = np.arctan2(np.linalg.norm(np.cross(pts[:-1], pts[1:]), axis=1),
                           np.einsum("ij,ij->i", pts[:-1], pts[1:]))
            assert np.abs(a - th0 / n).max() < 2e-15
            # all on the great circle through V_i, V_j
            nrm = np.cross(V[i], V[j])
            assert np.abs(pts @ nrm).max() < 1e-15
            e += 1
    assert e == 30


@pytest.mark.parametrize("n", [4, 6, 8, 20])
def test_icosahedral_symmetry(orc, n):
    # the grid is invariant (as a set) under the 60 rotations of the icosahedron
    d = orc.launch_dirs(n)
    rots = ico_rotations()
    assert len(rots) == 60
    for R in rots:
        W = d @ R.T
        G = W @ d.T
        assert np.abs(1.0 - G.max(axis=1)).max() < 1e-12


@pytest.mark.parametrize("n", [3, 4, 5, 6, 7, 8, 9, 10, 21])
def test_layer_sizes_and_innermost_cases(orc, n):
    """Layer a of a face has 3n - 9a points; innermost layer by n mod 3:
    one centre ray (n = 0 mod 3), three rays (n = 1), none (n = 2)."""
    d = orc.launch_dirs(n)
    per_face = (n - 1) * (n - 2) // 2
    sizes = []
    a = 1
    while n - 3 * a >= 0:
        sizes.append(3 * (n - 3 * a) if n - 3 * a > 0 else 1)
        a += 1
    assert sum(sizes) == per_face
    V = d[:12]
    faces = ico_faces(V)
    base = 12 + 30 * (n - 1)
    for f_i, f in enumerate(faces):
        pts = d[base + f_i * per_face: base + (f_i + 1) * per_face]
        cen = V[list(f)].sum(axis=0)
        cen /= np.linalg.norm(cen)
        # every interior point is inside the spherical triangle of its face
        A, B, Cc = V[list(f)]
        s = np.sign(np.linalg.det(np.stack([A, B, Cc])))
        for P, Q in ((A, B), (B, Cc), (Cc, A)):
            assert (s * (pts @ np.cross(P, Q)) > 0).all()
        start = sum(sizes[:-1])
        last = pts[start:]
        if n % 3 == 0:
            assert len(last) == 1 and np.abs(last[0] - cen).max() < 1e-15
        elif n % 3 == 1:
            assert len(last) == 3
            # three rays symmetric about the face centre
            ang = np.arccos(np.clip(last @ cen, -1, 1))
            assert np.ptp(ang) < 1e-12
        else:
            assert len(last) == 6
        # each ring is symmetric under the face's 3-fold rotation about its centre
        off = 0
        for m3 in sizes:
            ring = pts[off: off + m3]
            ang = np.arccos(np.clip(ring @ cen, -1, 1))
            if m3 >= 3:
                k = m3 // 3
                assert np.abs(ang[:k] - ang[k: 2 * k]).max() < 1e-12
                assert np.abs(ang[:k] - ang[2 * k:]).max() < 1e-12
                # eq. (1) on inner layers: along each side (corner b = 0, k, 2k
                # to the next corner) the points lie on one great circle at
                # equal angles
                for s_ in range(3):
                    side = np.concatenate([ring[s_ * k: (s_ + 1) * k], ring[((s_ + 1) % 3) * k][None]])
                    a_ = np.arctan2(np.linalg.norm(np.cross(side[:-1], side[1:]), axis=1),
                                    np.einsum("ij,ij->i", side[:-1], side[1:]))
                    assert np.ptp(a_) < 1e-14
                    nrm = np.cross(side[0], side[-1])
                    assert np.abs(side @ nrm).max() < 1e-15
            off += m3


OCTA_SIGNED_PERMS = [np.diag(sg)[list(pm)] for pm in
                     [(0, 1, 2), (0, 2, 1), (1, 0, 2), (1, 2, 0), (2, 0, 1), (2, 1, 0)]
                     for sg in [(a, b, c) for a in (1, -1) for b in (1, -1) for c in (1, -1)]]


def _same_set(P, Q, tol):
    assert P.shape == Q.shape
    d = np.abs(P[:, None, :] - Q[None, :, :]).max(axis=2)
    return d.min(axis=1).max() < tol and d.min(axis=0).max() < tol


@pytest.mark.parametrize("launch", [1, 2])
def test_equidistant_counts_norms_and_vertices(orc, launch):
    """Sec. II.A: 10 n^2 + 2 (icosahedron) or 4 n^2 + 2 (octahedron) unit
    directions; n = 1 gives the polyhedron's vertices."""
    per = 10 if launch == 1 else 4
    for n in range(1, 13):
        d = orc.launch_dirs(n, launch=launch)
        assert len(d) == orc.num_rays(n, launch) == per * n * n + 2
        assert np.abs(np.linalg.norm(d, axis=1) - 1.0).max() < 4.5e-16
    V = ico_vertex_set() if launch == 1 else octa_faces()[0]
    assert _same_set(orc.launch_dirs(1, launch=launch), V, 1e-15)


def test_equidistant_octahedron_n2_closed_form(orc):
    """n = 2 on the octahedron: the 6 axes and the 12 edge midpoints
    (+-1, +-1, 0)/sqrt(2) and permutations."""
    r = 1.0 / math.sqrt(2.0)
    mids = [p for p in ([a, b, 0.0] for a in (r, -r) for b in (r, -r))]
    mids = [np.array(m)[list(pm)] for m in mids for pm in [(0, 1, 2), (0, 2, 1), (2, 0, 1)]]
    want = np.concatenate([octa_faces()[0], np.array(mids)])
    assert _same_set(orc.launch_dirs(2, launch=2), want, 2e-16)


@pytest.mark.parametrize("launch,n", [(1, 7), (1, 12), (2, 9), (2, 14)])
def test_equidistant_points_are_equally_spaced_on_the_faces(orc, launch, n):
    """The defining property of equidistant division: centrally projected back
    onto the flat polyhedron faces, the face-interior points are exactly the
    barycentric lattice {(a, b, c)/n : a, b, c >= 1} and the edge points divide
    each edge chord into n equal parts."""
    d = orc.launch_dirs(n, launch=launch)
    nv, ne = (12, 30) if launch == 1 else (6, 12)
    V = d[:nv]  # the vertex rays come first (pinned as a set above)
    faces = [(i, j, k) for i in range(nv) for j in range(i + 1, nv) for k in range(j + 1, nv)
             if min(V[i] @ V[j], V[j] @ V[k], V[i] @ V[k]) > (0 if launch == 1 else -0.5)]
    # edges: adjacent vertex pairs i < j in lexicographic order, as documented
    edges = [(i, j) for i in range(nv) for j in range(i + 1, nv)
             if V[i] @ V[j] > (0 if launch == 1 else -0.5)]
    assert len(edges) == ne and len(faces) == (20 if launch == 1 else 8)
    E = d[nv: nv + ne * (n - 1)].reshape(ne, n - 1, 3)
    for (i, j), pts in zip(edges, E):
        # p ~ (1 - s) Vi + s Vj  =>  s = (p x Vi) . (Vj x Vi) / |Vj x Vi|^2 on the chord
        s = np.array([np.linalg.lstsq(np.stack([V[i], V[j] - V[i]], 1), p, rcond=None)[0]
                      for p in pts])
        s = s[:, 1] / s[:, 0]
        assert np.abs(s - np.arange(1, n) / n).max() < 1e-13
    F = d[nv + ne * (n - 1):].reshape(len(faces), (n - 1) * (n - 2) // 2, 3)
    want = sorted((a, b, n - a - b) for a in range(1, n) for b in range(1, n) if n - a - b >= 1)
    for pts in F:
        # the face the block belongs to: the one whose vertices span it positively
        lam = None
        for f in faces:
            M = V[list(f)].T
            L = np.linalg.solve(M, pts.T).T
            if (L > 0).all():
                lam = L / L.sum(axis=1, keepdims=True) * n
                break
        assert lam is not None
        got = sorted(tuple(int(round(x)) for x in row) for row in lam)
        assert np.abs(lam - np.round(lam)).max() < 1e-11
        cyc = {tuple(np.roll(w, k)) for w in want for k in range(3)}
        assert all(g in cyc for g in got) and len(set(got)) == len(want)


@pytest.mark.parametrize("launch,n", [(1, 6), (2, 7)])
def test_equidistant_symmetry(orc, launch, n):
    """The point set is invariant under the polyhedron's symmetry group (60
    rotations of the icosahedron; 48 signed permutations for the octahedron)
    and equals an independent lattice-and-project construction."""
    d = orc.launch_dirs(n, launch=launch)
    group = ico_rotations() if launch == 1 else OCTA_SIGNED_PERMS
    assert len(group) == (60 if launch == 1 else 48)
    for R in group[:: 5 if launch == 1 else 3]:
        assert _same_set(d @ R.T, d, 1e-14)
    if launch == 1:
        V = ico_vertex_set()
        ref = equidistant_grid(V, ico_faces(V), n)
    else:
        Vo, Fo = octa_faces()
        ref = equidistant_grid(Vo, Fo, n)
    assert _same_set(d, ref, 1e-14)


def test_equiangular_more_uniform_than_equidistant(orc):
    """Sec. II.B / Fig. 2: at the same ray count, equiangular division on the
    icosahedron is more uniform than equidistant division on the icosahedron,
    which is more uniform than equidistant division on the octahedron."""
    n = 21
    d = orc.launch_dirs(n)
    eq_ico = orc.launch_dirs(n, launch=1)
    assert len(eq_ico) == len(d) == 4412
    eq_oct = orc.launch_dirs(33, launch=2)   # 4 * 33^2 + 2 = 4358 rays
    assert len(eq_oct) == 4358

    def stats(P):
        a = nearest_angles(P)
        return a.std() / a.mean(), a.max() / a.min()

    cv_a, r_a = stats(d)
    cv_i, r_i = stats(eq_ico)
    cv_o, r_o = stats(eq_oct)
    assert cv_a < cv_i < cv_o
    assert r_a < r_i < r_o


def test_covering_radius_close_to_cone(orc):
    """Every direction should lie close to a ray.  The covering radius (the
    largest angle from any direction to its nearest ray) is compared with
    the cone half-angle theta_launch of eq. (4): it is about 1.155
    theta_launch for equiangular division, smaller than for equidistant
    division at the same n, so cones of half-angle theta_launch leave small
    gaps (one source of paths that SBR misses)."""
    n = 20
    d = orc.launch_dirs(n)
    V = ico_vertex_set()
    e = equidistant_grid(V, ico_faces(V), n)
    rng = np.random.default_rng(5)
    q = rng.normal(size=(200000, 3))
    q /= np.linalg.norm(q, axis=1, keepdims=True)

    def cover(P):
        best = np.full(len(q), -2.0)
        for s in range(0, len(q), 20000):
            best[s:s + 20000] = (q[s:s + 20000] @ P.T).max(axis=1)
        return np.arccos(np.clip(best, -1, 1)).max()

    thl = math.atan(2.0) / (math.sqrt(3.0) * n)
    ca, ce = cover(d), cover(e)
    assert ca < ce
    assert 1.0 < ca / thl < 1.17


def _dec_sin(x):
    getcontext().prec = 60
    X = Decimal(x)
    term, s, k = X, X, 1
    while abs(term) > Decimal(10) ** -58:
        term = -term * X * X / ((2 * k) * (2 * k + 1))
        s += term
        k += 1
    return s


def _dec_to_nearest_double(D):
    f = float(D)   # Decimal -> float conversion is correctly rounded
    return f


def test_trig_correctly_rounded(orc):
    rng = np.random.default_rng(11)
    xs = np.concatenate([rng.uniform(0, 1.2, 300), rng.uniform(0, 1e-3, 50)])
    for x in xs:
        assert orc.sin_cr(float(x)) == _dec_to_nearest_double(_dec_sin(float(x)))
    # acos: x = acos_cr(c) must be the nearest double to the true angle, i.e.
    # cos of its two neighbours brackets c on opposite sides.
    getcontext().prec = 60
    for c in rng.uniform(0.3, 1.0 - 1e-9, 300):
        t = orc.acos_cr(float(c))
        lo, hi = np.nextafter(t, 0), np.nextafter(t, 4)

        def dcos(v):
            X = Decimal(v)
            term, s, k = Decimal(1), Decimal(1), 1
            while abs(term) > Decimal(10) ** -58:
                term = -term * X * X / ((2 * k - 1) * (2 * k))
                s += term
                k += 1
            return s

        C_ = Decimal(float(c))
        # midpoints between t and its neighbours bracket the true angle
        m_lo = (Decimal(lo) + Decimal(t)) / 2
        m_hi = (Decimal(t) + Decimal(hi)) / 2
        assert dcos(m_lo) >= C_ >= dcos(m_hi)


def _face_rings(d, n, f_i):
    """Interior rings of face f_i (oracle ray order: a contiguous block per
    face, ring after ring, each of 3(n - 3a) points with its corners at
    positions 0, m, 2m)."""
    per_face = (n - 1) * (n - 2) // 2
    base = 12 + 30 * (n - 1) + f_i * per_face
    rings, off, a = [], 0, 1
    while n - 3 * a >= 1:
        m = n - 3 * a
        rings.append((m, d[base + off: base + off + 3 * m]))
        off += 3 * m
        a += 1
    return rings


@pytest.mark.parametrize("n", [4, 7, 10, 20])
def test_inner_corners_are_flat_face_parallelogram_completions(orc, n):
    """Eq. (2), Sec. II.B and Fig. 3b: every corner X of ring a+1 completes
    the parallelogram of its corner P^0 on ring a and the two ring-a points
    P^1, P^-1 next to it, X = P^1 + P^-1 - P^0, on the flat icosahedron face.
    The points are taken from the oracle's grid and centrally projected onto
    the face's plane here; the neighbours are found geometrically (ring 0 is
    the face's vertices and edge points)."""
    d = orc.launch_dirs(n)
    V = d[:12]
    faces = ico_faces(V)
    adj = V @ V.T > 0
    edges = [(i, j) for i in range(12) for j in range(i + 1, 12) if adj[i, j]]
    worst = 0.0
    for f_i, f in enumerate(faces):
        g = V[list(f)].sum(axis=0)

        def proj(p):
            return p / (p @ g)

        ring0 = [V[v] for v in f]
        for e_i, (i, j) in enumerate(edges):
            if i in f and j in f:
                ring0 += list(d[12 + e_i * (n - 1): 12 + (e_i + 1) * (n - 1)])
        prev_pts, prev_corners = np.array(ring0), V[list(f)]
        for m, ring in _face_rings(d, n, f_i):
            for s in range(3):
                X = ring[s * m]
                P0 = prev_corners[np.argmax(prev_corners @ X)]
                near = np.argsort(-(prev_pts @ P0))
                assert np.abs(prev_pts[near[0]] - P0).max() == 0.0
                P1, Pm = prev_pts[near[1]], prev_pts[near[2]]
                Y = proj(P1) + proj(Pm) - proj(P0)
                Y /= np.linalg.norm(Y)
                ang = np.arctan2(np.linalg.norm(np.cross(X, Y)), X @ Y)
                worst = max(worst, ang)
            prev_pts, prev_corners = ring, ring[[0, m, 2 * m]]
    # the same completion on the unit sphere instead of the flat face would
    # be off by about a tenth of the step angle
    assert worst < 1e-14, worst
