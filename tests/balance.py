"""Water-balance bookkeeping for the conservation pins, written from the
finite-volume reading of the discrete operator: control volumes
V_i = prod_l w_l h_l (w = 1/2 on a boundary of axis l), face areas
prod_{m != l} w_m h_m, arithmetic face averages of K*."""
import numpy as np


def volumes_and_weights(g):
    dim = g.dim
    hs = [g.L[l] / (g.n[l] - 1) for l in range(dim)]
    wl = []
    for l in range(dim):
        w = np.ones(g.n[l])
        w[0] = w[-1] = 0.5
        sh = [1] * dim
        sh[dim - 1 - l] = g.n[l]
        wl.append(w.reshape(sh))
    V = np.ones(g.shape)
    for l in range(dim):
        V = V * wl[l] * hs[l]
    return V, wl, hs


def dirichlet_inflow(g, psi, K, kinds, z):
    """Sum over faces between an unknown node i and a Dirichlet node b of
    A_f k_f (Phi_b - Phi_i) / h, Phi = psi + z (inflow positive)."""
    dim = g.dim
    shape = g.shape
    _, wl, hs = volumes_and_weights(g)
    phi = psi + z
    unk = ~kinds
    total = 0.0
    for l in range(dim):
        ax = dim - 1 - l
        area = np.ones(shape)
        for m in range(dim):
            if m != l:
                area = area * wl[m] * hs[m]
        for s in (-1, 1):
            nb_phi = np.roll(phi, -s, axis=ax)
            nb_K = np.roll(K, -s, axis=ax)
            nb_kind = np.roll(kinds, -s, axis=ax)
            valid = np.ones(shape, dtype=bool)
            idx = [slice(None)] * dim
            idx[ax] = -1 if s == 1 else 0
            valid[tuple(idx)] = False
            sel = unk & valid & nb_kind
            kf = 0.5 * (K + nb_K)
            total += np.sum((area * kf * (nb_phi - phi) / hs[l])[sel])
    return total


def drainage_outflow(g, K, kinds):
    """Free-drainage outflow through the bottom face: sum of A_z K*_i."""
    dim = g.dim
    _, wl, hs = volumes_and_weights(g)
    area = np.ones(g.shape)
    for m in range(dim - 1):
        area = area * wl[m] * hs[m]
    bottom = [slice(None)] * dim
    bottom[0] = 0
    bottom = tuple(bottom)
    return np.sum((area * K)[bottom][~kinds[bottom]])
