"""The largest grid the library takes: the 3-D Haverkamp block at 1025^3
nodes (1.077e9 nodes, just under the 2^31-node limit; a 76 GB workspace),
started unsaturated (psi0 = -0.3 - 0.7 z m) and moved by one V-cycle.
Step set-up and one red-black sweep are checked on sampled nodes: K* and g
against the oracle's laws, and every sampled update against the oracle's
pointwise solve applied to the point-update equation (eq. point-update:
f = g + sum_j m_ij psi_j + kappa psi, c = xi + kappa + m_ii) assembled from the
GPU's own inputs (red from the pre-sweep state, black from the new red values)."""
import dataclasses

import numpy as np
import pytest

import oracle
import paper_2606_04292_amd as rsl
from paper_2606_04292_amd import workloads as W
from tests.test_gpu_parity import TOL_SWEEP, say

pytestmark = pytest.mark.gpu


def test_largest_grid_sampled_setup_and_sweep():
    import torch
    assert torch.cuda.is_available()
    n = 1025
    w = W.config3(n)
    w = dataclasses.replace(w, psi0=None)
    w = dataclasses.replace(w, psi0=-0.3 - 0.7 * W.elevation(w.grid))
    say("max-size grid", n, "nodes", n ** 3)
    G = rsl.Grid(w)
    G.begin_step()
    G.vcycle()
    psin = G.get_state()[0].view(-1)
    psi0 = G.psi().view(-1)
    G.sweep(1)
    psi1 = G.psi().view(-1)
    K = G.field(rsl.FIELD_KSTAR).view(-1)
    g = G.field(rsl.FIELD_G).view(-1)
    torch.cuda.synchronize()
    G.close()
    del G
    law = w.law
    th, _, Kr, _, _ = oracle.law_fns(law)
    h = 1.0 / (n - 1)
    a = 1.0 / w.dt                 # the first step is BDF1
    rng = np.random.default_rng(31)
    ijk = rng.integers(1, n - 1, size=(4000, 3))       # unknown nodes (bottom face is Dirichlet)
    ijk[:200, 0] = 0                                    # some on the no-flux faces
    ijk[200:400, 1] = n - 1
    ijk[400:600, 2] = n - 1

    def lin(c):
        return c[..., 0] + n * (c[..., 1] + n * c[..., 2])

    def take(t, idx):
        return t[torch.as_tensor(idx.ravel(), device=t.device)].cpu().numpy().reshape(idx.shape)

    offs = np.array([[-1, 0, 0], [1, 0, 0], [0, -1, 0], [0, 1, 0], [0, 0, -1], [0, 0, 1]])
    nb = ijk[:, None, :] + offs[None, :, :]
    exists = np.all((nb >= 0) & (nb <= n - 1), axis=2)
    nbc = np.where(exists[..., None], nb, ijk[:, None, :])
    i0, inb = lin(ijk), lin(nbc)
    w_ax = np.where((ijk == 0) | (ijk == n - 1), 0.5, 1.0)            # control-volume fraction
    cf = np.where(exists, 1.0 / (2.0 * w_ax[:, offs.nonzero()[1]] * h * h), 0.0)
    Ki, Kn = take(K, i0), take(K, inb)
    gi = take(g, i0)
    p0, p0n, p1n = take(psi0, i0), take(psi0, inb), take(psi1, inb)
    ps = take(psin, i0)
    p1 = take(psi1, i0)
    # set-up: K* = Ks K_r(psi^n) and g = theta(psi^n)/tau + xi psi^n - (M z)_i
    want_K = np.array([law.Ks * Kr(x) for x in ps])
    assert np.all(np.abs(Ki - want_K) <= 1e-12 * np.abs(want_K))
    m = cf * (Ki[:, None] + Kn)
    side = np.array([0, 0, 0, 0, -1, 1])
    mz = (m * (-side * h)).sum(axis=1)
    want_g = np.array([th(x) * a for x in ps]) + law.xi * ps - mz
    assert np.abs(gi - want_g).max() <= TOL_SWEEP * np.abs(want_g).max()
    # the sweep: red nodes see the old black values, black nodes the new red ones
    red = (ijk.sum(axis=1) % 2) == 0
    pn = np.where(red[:, None], p0n, p1n)
    mii = m.sum(axis=1)
    kap = law.kappa * mii                                           # KAPPA_REL
    f = gi + (m * pn).sum(axis=1) + kap * p0
    c = law.xi + kap + mii
    want = np.array([oracle.local_solve(law, a, 0.0, c[q], f[q], p0[q], law.newton_iters)
                     for q in range(len(p0))])
    e_red = np.abs(p1[red] - want[red]).max() / np.abs(psi1.abs().max().item())
    e_black = np.abs(p1[~red] - want[~red]).max() / np.abs(psi1.abs().max().item())
    say("  sampled red rel", e_red, "black rel", e_black)
    assert e_red <= TOL_SWEEP and e_black <= TOL_SWEEP
