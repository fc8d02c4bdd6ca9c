"""Procedural reference shapes: an icosphere and articulated capsule figures.

No mesh library is available, so both are generated here. The capsule
figures are sampled as oriented point sets (positions + analytic normals) on
the union surface of their capsules; the method's hot path needs vertex
positions and normals only (Sec. 3, problem statement).
"""
import numpy as np


def icosphere(subdiv=4):
    """Unit icosphere by repeated midpoint subdivision.

    Returns (vertices [V,3] float64, faces [F,3] int64, edges [E,2] int64).
    subdiv=4 gives 2562 vertices, 5120 faces and 7680 edges.
    """
    t = (1.0 + 5.0 ** 0.5) / 2.0
    verts = [(-1, t, 0), (1, t, 0), (-1, -t, 0), (1, -t, 0),
             (0, -1, t), (0, 1, t), (0, -1, -t), (0, 1, -t),
             (t, 0, -1), (t, 0, 1), (-t, 0, -1), (-t, 0, 1)]
    faces = [(0, 11, 5), (0, 5, 1), (0, 1, 7), (0, 7, 10), (0, 10, 11),
             (1, 5, 9), (5, 11, 4), (11, 10, 2), (10, 7, 6), (7, 1, 8),
             (3, 9, 4), (3, 4, 2), (3, 2, 6), (3, 6, 8), (3, 8, 9),
             (4, 9, 5), (2, 4, 11), (6, 2, 10), (8, 6, 7), (9, 8, 1)]
    v = [np.array(p, dtype=np.float64) / np.linalg.norm(p) for p in verts]
    f = list(faces)
    for _ in range(subdiv):
        cache = {}

        def mid(a, b):
            key = (a, b) if a < b else (b, a)
            if key not in cache:
                m = v[a] + v[b]
                v.append(m / np.linalg.norm(m))
                cache[key] = len(v) - 1
            return cache[key]

        nf = []
        for a, b, c in f:
            ab, bc, ca = mid(a, b), mid(b, c), mid(c, a)
            nf += [(a, ab, ca), (b, bc, ab), (c, ca, bc), (ab, bc, ca)]
        f = nf
    V = np.array(v)
    F = np.array(f, dtype=np.int64)
    e = np.concatenate([F[:, [0, 1]], F[:, [1, 2]], F[:, [2, 0]]])
    e.sort(axis=1)
    E = np.unique(e, axis=0)
    return V, F, E


# --- articulated capsule figures -------------------------------------------
# A figure is a list of joints (name, parent index, rest position) and a list
# of capsules (segment end points, radius, driving joint index).

def _human():
    J = [  # name, parent, rest position (metres-ish)
        ("root", -1, (0.0, 0.95, 0.0)),
        ("spine", 0, (0.0, 1.02, 0.0)),
        ("neck", 1, (0.0, 1.40, 0.0)),
        ("head", 2, (0.0, 1.55, 0.0)),
        ("shoulder_l", 1, (0.19, 1.38, 0.0)),
        ("elbow_l", 4, (0.46, 1.38, 0.0)),
        ("shoulder_r", 1, (-0.19, 1.38, 0.0)),
        ("elbow_r", 6, (-0.46, 1.38, 0.0)),
        ("hip_l", 0, (0.10, 0.90, 0.0)),
        ("knee_l", 8, (0.10, 0.49, 0.0)),
        ("ankle_l", 9, (0.10, 0.07, 0.0)),
        ("hip_r", 0, (-0.10, 0.90, 0.0)),
        ("knee_r", 11, (-0.10, 0.49, 0.0)),
        ("ankle_r", 12, (-0.10, 0.07, 0.0)),
    ]
    C = [  # a, b, radius, joint
        ((-0.12, 0.93, 0.0), (0.12, 0.93, 0.0), 0.12, 0),    # pelvis
        ((0.0, 1.08, 0.0), (0.0, 1.30, 0.0), 0.15, 1),       # chest
        ((0.0, 1.42, 0.0), (0.0, 1.50, 0.0), 0.055, 2),      # neck
        ((0.0, 1.62, 0.01), (0.0, 1.71, 0.01), 0.10, 3),     # head
        ((0.21, 1.38, 0.0), (0.44, 1.38, 0.0), 0.052, 4),    # upper arm l
        ((0.48, 1.38, 0.0), (0.71, 1.38, 0.0), 0.042, 5),    # forearm l
        ((-0.21, 1.38, 0.0), (-0.44, 1.38, 0.0), 0.052, 6),  # upper arm r
        ((-0.48, 1.38, 0.0), (-0.71, 1.38, 0.0), 0.042, 7),  # forearm r
        ((0.10, 0.84, 0.0), (0.10, 0.52, 0.0), 0.075, 8),    # thigh l
        ((0.10, 0.46, 0.0), (0.10, 0.12, 0.0), 0.055, 9),    # shin l
        ((0.10, 0.04, -0.02), (0.10, 0.04, 0.15), 0.042, 10),  # foot l
        ((-0.10, 0.84, 0.0), (-0.10, 0.52, 0.0), 0.075, 11),   # thigh r
        ((-0.10, 0.46, 0.0), (-0.10, 0.12, 0.0), 0.055, 12),   # shin r
        ((-0.10, 0.04, -0.02), (-0.10, 0.04, 0.15), 0.042, 13),  # foot r
    ]
    return J, C


def _quadruped():
    J = [
        ("root", -1, (0.0, 0.80, 0.0)),
        ("chest", 0, (0.0, 0.80, 0.35)),
        ("neck", 1, (0.0, 0.88, 0.50)),
        ("head", 2, (0.0, 1.05, 0.68)),
        ("tail0", 0, (0.0, 0.82, -0.42)),
        ("tail1", 4, (0.0, 0.80, -0.70)),
        ("fl_hip", 1, (0.14, 0.72, 0.36)),
        ("fl_knee", 6, (0.14, 0.42, 0.36)),
        ("fr_hip", 1, (-0.14, 0.72, 0.36)),
        ("fr_knee", 8, (-0.14, 0.42, 0.36)),
        ("hl_hip", 0, (0.14, 0.72, -0.34)),
        ("hl_knee", 10, (0.14, 0.42, -0.34)),
        ("hr_hip", 0, (-0.14, 0.72, -0.34)),
        ("hr_knee", 12, (-0.14, 0.42, -0.34)),
    ]
    C = [
        ((0.0, 0.80, -0.35), (0.0, 0.80, 0.35), 0.17, 0),     # torso
        ((0.0, 0.86, 0.46), (0.0, 0.98, 0.62), 0.075, 2),     # neck
        ((0.0, 1.05, 0.68), (0.0, 1.02, 0.88), 0.085, 3),     # head
        ((0.0, 0.82, -0.44), (0.0, 0.81, -0.68), 0.04, 4),    # tail 0
        ((0.0, 0.80, -0.72), (0.0, 0.74, -0.98), 0.03, 5),    # tail 1
        ((0.14, 0.68, 0.36), (0.14, 0.45, 0.36), 0.06, 6),    # front left upper
        ((0.14, 0.39, 0.36), (0.14, 0.05, 0.38), 0.045, 7),   # front left lower
        ((-0.14, 0.68, 0.36), (-0.14, 0.45, 0.36), 0.06, 8),
        ((-0.14, 0.39, 0.36), (-0.14, 0.05, 0.38), 0.045, 9),
        ((0.14, 0.68, -0.34), (0.14, 0.45, -0.34), 0.065, 10),
        ((0.14, 0.39, -0.34), (0.14, 0.05, -0.32), 0.045, 11),
        ((-0.14, 0.68, -0.34), (-0.14, 0.45, -0.34), 0.065, 12),
        ((-0.14, 0.39, -0.34), (-0.14, 0.05, -0.32), 0.045, 13),
    ]
    return J, C


FIGURES = {"human": _human, "quadruped": _quadruped}


def _seg_dist(P, a, b):
    ab = b - a
    t = np.clip(((P - a) @ ab) / (ab @ ab), 0.0, 1.0)
    return np.linalg.norm(P - (a + t[:, None] * ab), axis=1)


def _sample_capsule(rng, a, b, r, n):
    """n area-uniform samples (positions, outward normals) on one capsule."""
    a = np.asarray(a, float)
    b = np.asarray(b, float)
    ax = b - a
    h = np.linalg.norm(ax)
    u = ax / h
    tmp = np.array([1.0, 0, 0]) if abs(u[0]) < 0.9 else np.array([0, 1.0, 0])
    e1 = np.cross(u, tmp)
    e1 /= np.linalg.norm(e1)
    e2 = np.cross(u, e1)
    a_cyl = 2 * np.pi * r * h
    a_sph = 4 * np.pi * r * r
    on_cyl = rng.random(n) < a_cyl / (a_cyl + a_sph)
    P = np.empty((n, 3))
    N = np.empty((n, 3))
    k = on_cyl.sum()
    phi = rng.random(k) * 2 * np.pi
    s = rng.random(k) * h
    rad = np.cos(phi)[:, None] * e1 + np.sin(phi)[:, None] * e2
    P[on_cyl] = a + s[:, None] * u + r * rad
    N[on_cyl] = rad
    m = n - k
    d = rng.normal(size=(m, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    cap = np.where(((d @ u) > 0)[:, None], b, a)
    P[~on_cyl] = cap + r * d
    N[~on_cyl] = d
    return P, N


def capsule_figure(kind, n, rng, oversample=1.6):
    """n oriented samples on the union surface of a capsule figure.

    Samples lying inside another capsule are rejected, so the set describes
    the outer surface only. Returns (P [n,3], N [n,3], owner capsule [n]).
    """
    J, C = FIGURES[kind]()
    areas = np.array([2 * np.pi * r * np.linalg.norm(np.subtract(b, a)) + 4 * np.pi * r * r
                      for a, b, r, _ in C])
    Ps, Ns, Os = [], [], []
    total = 0
    while total < n:
        m = int((n - total) * oversample) + 64
        counts = rng.multinomial(m, areas / areas.sum())
        for ci, (a, b, r, _) in enumerate(C):
            if counts[ci] == 0:
                continue
            P, Nn = _sample_capsule(rng, a, b, r, counts[ci])
            keep = np.ones(len(P), bool)
            for cj, (a2, b2, r2, _) in enumerate(C):
                if cj != ci:
                    keep &= _seg_dist(P, np.asarray(a2, float), np.asarray(b2, float)) > r2 * 0.999
            Ps.append(P[keep])
            Ns.append(Nn[keep])
            Os.append(np.full(keep.sum(), ci))
            total += keep.sum()
    P = np.concatenate(Ps)
    N = np.concatenate(Ns)
    O = np.concatenate(Os)
    perm = rng.permutation(len(P))[:n]
    return P[perm], N[perm], O[perm]
