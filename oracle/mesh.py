"""Oracle mesh: Kuhn-cube tetrahedral meshes, topology and DoF numbering.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import this module.

The paper works on a tetrahedral complex of nodes, edges, faces and tets
(Sec. III-A, the mesh complex K = {N, E, F, T}).  It does not fix any mesh; the
workloads use a unit cube split into N^3 hexahedra with 6 tets each (the Kuhn
split along the main diagonal), which is conforming.

Conventions (shared by the oracle and the product only as a written
convention, not as code):
  * every tet stores its 4 global vertex ids sorted ascending;
  * edges are sorted vertex pairs, numbered in lexicographic order;
  * faces are sorted vertex triples, numbered in lexicographic order;
  * local edges of a tet: (0,1),(0,2),(0,3),(1,2),(1,3),(2,3);
  * local faces of a tet: (0,1,2),(0,1,3),(0,2,3),(1,2,3);
  * nbr[t, m] is the tet across the face opposite local vertex m (-1 = boundary).
"""
import itertools
import numpy as np

LOCAL_EDGES = [(0, 1), (0, 2), (0, 3), (1, 2), (1, 3), (2, 3)]
LOCAL_FACES = [(0, 1, 2), (0, 1, 3), (0, 2, 3), (1, 2, 3)]


class Mesh:
    """Plain container; every array is numpy."""


def kuhn_cube(N, L=1.0):
    """Vertices and tets of the N^3 Kuhn-split cube of side L.

    Vertex (i,j,l) has id i + (N+1)(j + (N+1) l) and position (i,j,l) L/N.
    Hex h = i + N (j + N l); for each permutation pi of the axes (in
    lexicographic order) tet 6h+p walks v0=(i,j,l), v0+e_pi0, +e_pi1, +e_pi2.
    """
    n1 = N + 1
    ii, jj, ll = np.meshgrid(np.arange(n1), np.arange(n1), np.arange(n1), indexing="ij")
    xyz = np.zeros((n1 ** 3, 3))
    vid = ii + n1 * (jj + n1 * ll)
    xyz[vid.ravel(), 0] = ii.ravel() * L / N
    xyz[vid.ravel(), 1] = jj.ravel() * L / N
    xyz[vid.ravel(), 2] = ll.ravel() * L / N
    tets = []
    perms = list(itertools.permutations(range(3)))
    for l in range(N):
        for j in range(N):
            for i in range(N):
                for p in perms:
                    c = [i, j, l]
                    vs = [c[0] + n1 * (c[1] + n1 * c[2])]
                    for ax in p:
                        c[ax] += 1
                        vs.append(c[0] + n1 * (c[1] + n1 * c[2]))
                    tets.append(sorted(vs))
    return xyz, np.array(tets, dtype=np.int64)


def build(xyz, tets, order):
    """Topology, geometry and DoF maps of a tet mesh (order k = 1 or 2).

    DoF numbering (natural order, the one every exported vector uses):
      W1, k=1: global edge id.
      W1, k=2: 2*edge + 0 -> Q = R^_2(3,l_lo) on (lo,hi) [higher multi-index on
               the lower vertex], 2*edge + 1 -> Q on the higher vertex;
               2*E + 2*face + 0 -> face (a,b,c) function 3 l_c W_ab,
               2*E + 2*face + 1 -> 3 l_b W_ac   (3 l_a W_bc is the dropped one).
      W2, k=1: face id.  k=2: 3*face + {0,1,2} -> (4 l_x - 1) W_abc with x = a,b,c;
               3*F + 3*tet + {0,1,2} -> 4 l_d W_f for local faces f = 0,1,2.
      W0, k=1: vertex id.  k=2: vertex id, then V + edge.
    """
    m = Mesh()
    m.xyz = np.asarray(xyz, dtype=np.float64)
    tets = np.sort(np.asarray(tets, dtype=np.int64), axis=1)
    m.tets = tets
    m.order = order
    nt = len(tets)
    nv = len(xyz)
    m.nv, m.nt = nv, nt

    # edges
    e_all = np.stack([tets[:, [a, b]] for a, b in LOCAL_EDGES], axis=1)  # (nt,6,2)
    ekey = e_all[..., 0] * nv + e_all[..., 1]
    uniq_e, tet_edge = np.unique(ekey.ravel(), return_inverse=True)
    m.edges = np.stack([uniq_e // nv, uniq_e % nv], axis=1)
    m.tet_edge = tet_edge.reshape(nt, 6)
    m.ne = len(uniq_e)

    # faces
    f_all = np.stack([tets[:, list(f)] for f in LOCAL_FACES], axis=1)  # (nt,4,3)
    fkey = (f_all[..., 0] * nv + f_all[..., 1]) * nv + f_all[..., 2]
    uniq_f, tet_face = np.unique(fkey.ravel(), return_inverse=True)
    m.faces = np.stack([uniq_f // (nv * nv), (uniq_f // nv) % nv, uniq_f % nv], axis=1)
    m.tet_face = tet_face.reshape(nt, 4)
    m.nf = len(uniq_f)

    # face -> incident tets, neighbours across the face opposite local vertex v
    # local face index of the face opposite vertex v is 3 - v
    face_tets = [[] for _ in range(m.nf)]
    for t in range(nt):
        for lf in range(4):
            face_tets[m.tet_face[t, lf]].append(t)
    m.face_ntet = np.array([len(x) for x in face_tets])
    assert m.face_ntet.max() <= 2
    nbr = -np.ones((nt, 4), dtype=np.int64)
    for t in range(nt):
        for v in range(4):
            f = m.tet_face[t, 3 - v]
            others = [u for u in face_tets[f] if u != t]
            if others:
                nbr[t, v] = others[0]
    m.nbr = nbr

    # boundary entities (PEC walls, Sec. II Dirichlet condition)
    bface = m.face_ntet == 1
    m.bface = bface
    bedge = np.zeros(m.ne, dtype=bool)
    bvert = np.zeros(nv, dtype=bool)
    ekey_sorted = m.edges[:, 0] * nv + m.edges[:, 1]
    for f in np.nonzero(bface)[0]:
        a, b, c = m.faces[f]
        bvert[[a, b, c]] = True
        for p, q in ((a, b), (a, c), (b, c)):
            bedge[np.searchsorted(ekey_sorted, p * nv + q)] = True
    m.bedge, m.bvert = bedge, bvert

    # geometry: lambda(r) = A^{-1} [r; 1], A columns [x_m; 1]
    X = m.xyz[tets]  # (nt,4,3)
    Amat = np.concatenate([np.transpose(X, (0, 2, 1)), np.ones((nt, 1, 4))], axis=1)  # (nt,4,4)
    Ainv = np.linalg.inv(Amat)  # rows m: [grad_m (3), a_m]
    m.grad = Ainv[:, :, :3].copy()  # (nt,4,3)
    m.aff = Ainv[:, :, 3].copy()  # (nt,4)
    m.vol = np.abs(np.linalg.det(X[:, 1:] - X[:, :1])) / 6.0

    # DoF maps
    E, F = m.ne, m.nf
    if order == 1:
        m.n0, m.n1, m.n2 = nv, E, F
        m.map1 = m.tet_edge.copy()
        m.map2 = m.tet_face.copy()
        m.map0 = tets.copy()
        m.int1 = ~bedge
        m.int0 = ~bvert
    elif order == 2:
        m.n0, m.n1, m.n2 = nv + E, 2 * E + 2 * F, 3 * F + 3 * nt
        map1 = np.zeros((nt, 20), dtype=np.int64)
        for le in range(6):
            map1[:, 2 * le] = 2 * m.tet_edge[:, le]
            map1[:, 2 * le + 1] = 2 * m.tet_edge[:, le] + 1
        for lf in range(4):
            map1[:, 12 + 2 * lf] = 2 * E + 2 * m.tet_face[:, lf]
            map1[:, 12 + 2 * lf + 1] = 2 * E + 2 * m.tet_face[:, lf] + 1
        m.map1 = map1
        map2 = np.zeros((nt, 15), dtype=np.int64)
        for lf in range(4):
            for x in range(3):
                map2[:, 3 * lf + x] = 3 * m.tet_face[:, lf] + x
        for x in range(3):
            map2[:, 12 + x] = 3 * F + 3 * np.arange(nt) + x
        m.map2 = map2
        m.map0 = np.concatenate([tets, nv + m.tet_edge], axis=1)
        int1 = np.ones(m.n1, dtype=bool)
        int1[: 2 * E] = np.repeat(~bedge, 2)
        int1[2 * E:] = np.repeat(~bface, 2)
        m.int1 = int1
        m.int0 = np.concatenate([~bvert, ~bedge])
    else:
        raise ValueError("order must be 1 or 2")
    m.N1_int = int(m.int1.sum())
    m.N0_int = int(m.int0.sum())
    return m


def cube_mesh(N, order, L=1.0):
    xyz, tets = kuhn_cube(N, L)
    m = build(xyz, tets, order)
    m.N, m.L = N, L
    return m


def locate_kuhn(m, pos):
    """Point location on a Kuhn cube: the hex from floor(r N / L) (clamped), then
    among its 6 tets the one with the largest min_m lambda_m (ties: smallest id)."""
    N, L = m.N, m.L
    pos = np.atleast_2d(np.asarray(pos, dtype=np.float64))
    idx = np.clip(np.floor(pos * N / L).astype(np.int64), 0, N - 1)
    h = idx[:, 0] + N * (idx[:, 1] + N * idx[:, 2])
    cand = 6 * h[:, None] + np.arange(6)[None, :]  # (P,6), ascending ids
    lam = m.aff[cand] + np.einsum("pqmk,pk->pqm", m.grad[cand], pos)
    mn = lam.min(axis=2)
    return cand[np.arange(len(pos)), np.argmax(mn, axis=1)]  # argmax: first (smallest id) on ties


def locate_brute(m, pos):
    """Point location by checking every tet (small meshes only)."""
    pos = np.atleast_2d(pos)
    lam = m.aff[None, :, :] + np.einsum("tmk,pk->ptm", m.grad, pos)
    mn = lam.min(axis=2)
    return np.argmax(mn, axis=1)  # argmax returns the first (smallest id) on ties
