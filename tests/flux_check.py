"""Net flux of a W2 field out of every tet: the part of its discrete divergence that needs no W3 basis.

B = sum_l b_l W2_l with W2_l = Q_l(lambda) 2(l_a grad l_b x grad l_c + cyclic) (Appendix, face
functions).  The flux out of face m of tet T is the integral of B . n over it, with the outward
normal n = -grad l_m / |grad l_m| and area 3 V |grad l_m|: -3 V times the face mean of
B . grad l_m.  Each face mean uses a collapsed 4 x 4 Gauss-Legendre rule on the triangle, exact for
the degrees of the order-1 and order-2 face functions.  Faraday's law keeps B solenoidal
(Sec. III-A: b changes by K e, and the divergence of a curl is zero), so from b = 0 every tet's net
flux stays at rounding level.
"""
import numpy as np

from oracle import basis


def tet_net_flux(m, b):
    """Per tet: the net outward flux of B, and the sum of the absolute face fluxes (its scale)."""
    _, _, f2, q2, _ = basis.c_tables(m.order)
    u, wu = basis.gauss_legendre01(4)
    g = m.grad  # (nt, 4, 3): grad lambda_m of each tet
    bl = np.asarray(b)[m.map2]  # (nt, n2 local)
    cr = {(i, j): np.cross(g[:, i], g[:, j]) for i in range(4) for j in range(4) if i != j}
    net = np.zeros(m.nt)
    tot = np.zeros(m.nt)
    for fm in range(4):
        o = [x for x in range(4) if x != fm]
        mean = np.zeros(m.nt)
        for ua, wa in zip(u, wu):
            for ub, wb in zip(u, wu):
                lam = np.zeros(4)
                lam[o[0]], lam[o[1]], lam[o[2]] = ua, ub * (1 - ua), (1 - ua) * (1 - ub)
                B = np.zeros((m.nt, 3))
                for l, (a, bb, c) in enumerate(f2):
                    Q = q2[l, 0] + q2[l, 1:] @ lam
                    W = 2 * (lam[a] * cr[(bb, c)] + lam[bb] * cr[(c, a)] + lam[c] * cr[(a, bb)])
                    B += (bl[:, l] * Q)[:, None] * W
                mean += 2 * wa * wb * (1 - ua) * np.einsum("tk,tk->t", B, g[:, fm])
        flux = -3 * m.vol * mean
        net += flux
        tot += np.abs(flux)
    return net, tot


def relative_net_flux(m, b):
    net, tot = tet_net_flux(m, b)
    return float(np.linalg.norm(net) / max(np.linalg.norm(tot), 1e-300))
