"""Pins of the oracle's mesh, simulation of simplicity and extraction.

Each check compares the oracle with something it does not compute itself:
the prism split as the paper lists it (Sec. III-C), a generic symbolic
expansion of the perturbed determinants (Sec. III-F), Lemma 1, the
Poincare-index/winding-number identity, and the closed-form critical path of a
translating radial vortex.
"""
import itertools
import math
from fractions import Fraction

import numpy as np
import pytest

import synthfields


# ---------------------------------------------------------------- brute force
def gid(H, W, x, y, t):
    return (t * H + y) * W + x


def brute_tets(H, W, T):
    """Tetrahedra of the space-time mesh, literally from Sec. III-C: each quad
    is split into two triangles, each triangle (vertices a<b<c by spatial
    index) is extruded over [t, t+1] and split into (a_t,b_t,c_t,c_t+1),
    (a_t,b_t,b_t+1,c_t+1), (a_t,a_t+1,b_t+1,c_t+1)."""
    tets = []
    for t in range(T - 1):
        for y in range(H - 1):
            for x in range(W - 1):
                for tri in (((x, y), (x + 1, y), (x + 1, y + 1)),
                            ((x, y), (x, y + 1), (x + 1, y + 1))):
                    a, b, c = sorted(tri, key=lambda p: p[1] * W + p[0])
                    g = lambda p, tt: gid(H, W, p[0], p[1], tt)
                    tets.append((g(a, t), g(b, t), g(c, t), g(c, t + 1)))
                    tets.append((g(a, t), g(b, t), g(b, t + 1), g(c, t + 1)))
                    tets.append((g(a, t), g(a, t + 1), g(b, t + 1), g(c, t + 1)))
    return tets


def brute_faces(H, W, T):
    faces = set()
    for tet in brute_tets(H, W, T):
        for f in itertools.combinations(sorted(tet), 3):
            faces.add(f)
    for t in range(T):  # slice triangles (the only faces when T == 1)
        for y in range(H - 1):
            for x in range(W - 1):
                for tri in (((x, y), (x + 1, y), (x + 1, y + 1)),
                            ((x, y), (x, y + 1), (x + 1, y + 1))):
                    faces.add(tuple(sorted(gid(H, W, p[0], p[1], t) for p in tri)))
    return faces


def typed_faces(ora, H, W, T):
    out = {}
    for t in range(T):
        for y in range(H):
            for x in range(W):
                for f in range(12):
                    vs = ora.face_vertices(f)
                    if all(x + dx < W and y + dy < H and t + dt < T for dx, dy, dt in vs):
                        tri = tuple(gid(H, W, x + dx, y + dy, t + dt) for dx, dy, dt in vs)
                        out[(gid(H, W, x, y, t), f)] = tri
    return out


# ---------------------------------------------------- generic symbolic SoS
def _poly_mul(a, b):
    out = {}
    for ea, ca in a.items():
        for eb, cb in b.items():
            out[ea + eb] = out.get(ea + eb, 0) + ca * cb
    return out


def _poly_sub(a, b):
    out = dict(a)
    for e, c in b.items():
        out[e] = out.get(e, 0) - c
    return out


def generic_det_sign(up, vp, gp, uq, vq, gq):
    """Sign of det(p~, q~) with u_g + eps^(2^(2g+1)), v_g + eps^(2^(2g)):
    expand the polynomial in eps and take the first nonzero coefficient."""
    Up = {0: up, 2 ** (2 * gp + 1): 1}
    Vp = {0: vp, 2 ** (2 * gp): 1}
    Uq = {0: uq, 2 ** (2 * gq + 1): 1}
    Vq = {0: vq, 2 ** (2 * gq): 1}
    d = _poly_sub(_poly_mul(Up, Vq), _poly_mul(Vp, Uq))
    for e in sorted(d):
        if d[e] != 0:
            return 1 if d[e] > 0 else -1
    return 0


def generic_crossed(U, V, tri):
    a, b, c = tri
    s1 = generic_det_sign(U[a], V[a], a, U[b], V[b], b)
    s2 = generic_det_sign(U[b], V[b], b, U[c], V[c], c)
    s3 = generic_det_sign(U[c], V[c], c, U[a], V[a], a)
    return (s1 == s2 == s3), s1


SHAPES = [(2, 2, 1), (3, 3, 2), (4, 3, 3), (3, 5, 2), (2, 4, 4)]


@pytest.mark.parametrize("H,W,T", SHAPES)
def test_typed_faces_equal_prism_split(ora, H, W, T):
    bf = brute_faces(H, W, T)
    tf = typed_faces(ora, H, W, T)
    assert len(set(tf.values())) == len(tf), "a face is listed twice"
    assert set(tf.values()) == bf


def test_incident_face_count_36(ora):
    H, W, T = 5, 6, 4
    bf = brute_faces(H, W, T)
    for (x, y, t) in [(2, 2, 1), (3, 2, 2), (1, 3, 1)]:
        v = gid(H, W, x, y, t)
        inc = {f for f in bf if v in f}
        assert len(inc) == 36
        nb = ora.incident_faces(H, W, T, x, y, t)
        assert len(nb) == 36
        got = {tuple(sorted((int(a), int(b), v))) for a, b in nb}
        assert got == inc
    # boundary vertices: the oracle agrees with brute force everywhere
    for t in range(T):
        for y in range(H):
            for x in range(W):
                v = gid(H, W, x, y, t)
                n = sum(1 for f in bf if v in f)
                assert len(ora.incident_faces(H, W, T, x, y, t)) == n


def test_sos_edge_matches_generic_expansion(ora):
    rng = np.random.default_rng(5)
    vals = [-2, -1, 0, 1, 2]
    for up, vp, uq, vq in itertools.product(vals, repeat=4):
        assert ora.lib().cpo_sos_edge(up, vp, uq, vq) == generic_det_sign(up, vp, 3, uq, vq, 7)
    for _ in range(4000):
        up, vp, uq, vq = (int(z) for z in rng.integers(-(1 << 24), 1 << 24, 4))
        if rng.random() < 0.3:
            vq = up * vq // max(abs(up), 1) if up else 0
        assert ora.lib().cpo_sos_edge(up, vp, uq, vq) == generic_det_sign(up, vp, 1, uq, vq, 2)


@pytest.mark.parametrize("H,W,T", SHAPES)
@pytest.mark.parametrize("seed", [0, 1, 2])
def test_extraction_matches_generic_sos(ora, H, W, T, seed):
    rng = np.random.default_rng(seed * 100 + H * 10 + W)
    U = rng.integers(-2, 3, (T, H, W)).astype(np.int32)
    V = rng.integers(-2, 3, (T, H, W)).astype(np.int32)
    Uf, Vf = U.ravel().tolist(), V.ravel().tolist()
    tf = typed_faces(ora, H, W, T)
    expect = []
    for (g, f), tri in sorted(tf.items()):
        cr, s = generic_crossed(Uf, Vf, tri)
        if cr:
            expect.append(((g * 12 + f) << 1) | (1 if s > 0 else 0))
    got = ora.extract_fixed(U, V)
    assert got.tolist() == sorted(expect)


def test_general_position_equals_plain_inside_test(ora):
    """Without zero determinants the SoS test is the plain sign test of the
    inside predicate (eq. inside-test)."""
    rng = np.random.default_rng(11)
    H, W, T = 6, 7, 3
    U = rng.integers(-1000, 1000, (T, H, W)).astype(np.int32)
    V = rng.integers(-1000, 1000, (T, H, W)).astype(np.int32)
    Uf, Vf = U.ravel().tolist(), V.ravel().tolist()
    got = set((ora.extract_fixed(U, V) >> 1).tolist())
    for (g, f), (a, b, c) in typed_faces(ora, H, W, T).items():
        d1 = Uf[a] * Vf[b] - Vf[a] * Uf[b]
        d2 = Uf[b] * Vf[c] - Vf[b] * Uf[c]
        d3 = Uf[c] * Vf[a] - Vf[c] * Uf[a]
        if 0 in (d1, d2, d3):
            continue
        plain = (d1 > 0 and d2 > 0 and d3 > 0) or (d1 < 0 and d2 < 0 and d3 < 0)
        assert plain == ((g * 12 + f) in got)


@pytest.mark.parametrize("seed", range(6))
def test_lemma1_zero_or_two_faces_per_tet(ora, seed):
    """Lemma 1: the zero set meets a tetrahedron's boundary in 0 or 2 points;
    checked on highly degenerate fields with values in {-1, 0, 1}."""
    rng = np.random.default_rng(seed)
    H, W, T = 5, 4, 4
    U = rng.integers(-1, 2, (T, H, W)).astype(np.int32)
    V = rng.integers(-1, 2, (T, H, W)).astype(np.int32)
    crossed = set((ora.extract_fixed(U, V) >> 1).tolist())
    tf = typed_faces(ora, H, W, T)
    tri2code = {tri: g * 12 + f for (g, f), tri in tf.items()}
    for tet in brute_tets(H, W, T):
        n = sum(1 for f in itertools.combinations(sorted(tet), 3) if tri2code[f] in crossed)
        assert n in (0, 2), tet
    # the oracle's own tetrahedron walk agrees
    field = np.stack([U, V]).astype(np.float32)
    bad, _ = ora.tracks(field, 0)
    assert bad == 0


def test_interior_faces_shared_by_two_tets():
    H, W, T = 4, 4, 3
    cnt = {}
    for tet in brute_tets(H, W, T):
        for f in itertools.combinations(sorted(tet), 3):
            cnt[f] = cnt.get(f, 0) + 1
    assert set(cnt.values()) <= {1, 2}
    assert sum(1 for v in cnt.values() if v == 2) > 0


def _winding(u, v):
    """Winding number of the PL field along the grid boundary (CCW)."""
    H, W = u.shape
    path = [(x, 0) for x in range(W)] + [(W - 1, y) for y in range(1, H)] + \
           [(x, H - 1) for x in range(W - 2, -1, -1)] + [(0, y) for y in range(H - 2, -1, -1)]
    tot = 0.0
    for (x1, y1), (x2, y2) in zip(path, path[1:]):
        a = (float(u[y1, x1]), float(v[y1, x1]))
        b = (float(u[y2, x2]), float(v[y2, x2]))
        tot += math.atan2(a[0] * b[1] - a[1] * b[0], a[0] * b[0] + a[1] * b[1])
    return tot / (2 * math.pi)


def test_poincare_index_sum_equals_boundary_winding(ora):
    f, _ = synthfields.workload(0)
    f = f.numpy()
    k, _, _ = ora.params(f, 1e-2)
    F = ora.to_fixed(f, k)
    T, H, W = F.shape[1:]
    codes = ora.extract(f, k)
    orient = {}
    for ft in (0, 1):
        (ax, ay, _), (bx, by, _), (cx, cy, _) = ora.face_vertices(ft)
        orient[ft] = np.sign((bx - ax) * (cy - ay) - (by - ay) * (cx - ax))
    for t in range(T):
        idx = 0
        for c in codes.tolist():
            g, ft, s = (c >> 1) // 12, (c >> 1) % 12, c & 1
            if ft < 2 and g // (H * W) == t:
                idx += (1 if s else -1) * orient[ft]
        w = _winding(F[0, t].astype(np.int64), F[1, t].astype(np.int64))
        assert abs(w - round(w)) < 1e-6
        assert idx == round(w), (t, idx, w)


def _seg_dist(p, q):
    """Distance from the origin to segment pq (2D)."""
    px, py = p
    qx, qy = q
    dx, dy = qx - px, qy - py
    L = dx * dx + dy * dy
    s = 0.0 if L == 0 else max(0.0, min(1.0, -(px * dx + py * dy) / L))
    return math.hypot(px + s * dx, py + s * dy)


@pytest.mark.parametrize("trial", range(6))
def test_single_vortex_faces_equal_analytic_path(ora, trial):
    """A radial vortex has values alpha_i J (x_i - c(t_i)) with alpha_i of one
    sign, so a face is crossed exactly when 0 lies in conv{x_i - c(t_i)}, i.e.
    when the straight space-time path c(t) = c0 + s t crosses it."""
    rng = np.random.default_rng(100 + trial)
    H, W, T = 24, 26, 6
    while True:
        c0 = (Fraction(int(rng.integers(8 * 64, 16 * 64)), 64), Fraction(int(rng.integers(8 * 64, 14 * 64)), 64))
        s = (Fraction(int(rng.integers(-32, 33)), 64), Fraction(int(rng.integers(-32, 33)), 64))
        ok = True
        expect = set()
        for t in range(T):
            for y in range(H):
                for x in range(W):
                    for ft in range(12):
                        vs = ora.face_vertices(ft)
                        if not all(x + dx < W and y + dy < H and t + dt < T for dx, dy, dt in vs):
                            continue
                        d = [(x + dx - c0[0] - s[0] * (t + dt), y + dy - c0[1] - s[1] * (t + dt))
                             for dx, dy, dt in vs]
                        df = [(float(a), float(b)) for a, b in d]
                        if min(_seg_dist(df[i], df[(i + 1) % 3]) for i in range(3)) < 1e-3:
                            ok = False
                            break
                        dets = [d[i][0] * d[(i + 1) % 3][1] - d[i][1] * d[(i + 1) % 3][0] for i in range(3)]
                        if all(z > 0 for z in dets) or all(z < 0 for z in dets):
                            expect.add(gid(H, W, x, y, t) * 12 + ft)
                    if not ok:
                        break
                if not ok:
                    break
            if not ok:
                break
        if ok:
            break
    gam = float(rng.uniform(0.5, 2.0) * rng.choice([-1, 1]))
    params = (np.array([[float(c0[0]), float(c0[1])]]), np.array([[float(s[0]), float(s[1])]]),
              np.array([gam]), np.array([float(rng.uniform(3, 6))]))
    f, _ = synthfields.vortex_field(H, W, T, 1, seed=0, noise=0.0, params=params)
    f = f.numpy()
    k, _, _ = ora.params(f, 1e-2)
    got = ora.extract(f, k)
    assert set((got >> 1).tolist()) == expect
    assert len(expect) > 0
    # slice crossings have Poincare index +1 (a centre)
    for c in got.tolist():
        ft = (c >> 1) % 12
        if ft < 2:
            orient = 1 if ft == 0 else -1
            assert (1 if c & 1 else -1) * orient == 1
    bad, ntr = ora.tracks(f, k)
    assert bad == 0 and ntr == 1
