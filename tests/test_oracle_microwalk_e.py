"""Oracle pin for MicroWalk-E (Sec. III-B): walks on an expanded cube that
holds conductors, against an independent absorbing-chain solve.

By Theorem 1 the exit distribution of Alg. 3 is that of the absorbing Markov
chain of the lattice.  In an expanded cube the chain has more absorbing
states: interior nodes inside a conductor (closed box) or at/beyond a grounded
window face end the walk there, and a link from a free node into such a node
is shortened to the fraction theta of its length at which it meets the object
(code rint(code / theta), theta >= 1/16).  The pin builds that chain in numpy
with closed-form thetas (axis-aligned faces) and solves it with a sparse LU;
the oracle's walks (bisection thetas, integer thresholds) must follow its
distribution over boundary nodes and absorbing nets, and its mean step count
must match the chain's E(tau) (Eq. 11 with absorbing interior nodes).
"""
import numpy as np
import pytest

import workloads as W
from oracle import pins

D, N = W.DIRICHLET, W.NEUMANN

CASES = {
    # grounded -x face through the cube, one conductor, a dielectric box and
    # a layer interface
    "face_and_conductor": dict(
        cond=[[0.62, 1.75, 1.52, 0.93, 2.33, 2.07]], nets=[0],
        diel=[[0.1, 1.3, 1.9, 0.5, 2.1, 2.8]], diel_eps=[7.0],
        layer_z0=[0.0, 2.22], layer_eps=[3.9, 2.7],
        bc=(D, N, N, N, N, N), centre=(0.4, 2.0, 2.0), R=0.6, n=8),
    # two conductors of different nets on opposite sides, grounded +z face,
    # high-contrast inclusion
    "two_conductors": dict(
        cond=[[2.31, 1.63, 1.7, 2.57, 2.49, 2.27], [1.2, 1.55, 1.58, 1.47, 2.21, 2.35]], nets=[0, 1],
        diel=[[1.66, 1.5, 1.5, 2.05, 1.95, 2.2]], diel_eps=[25.0],
        layer_z0=[0.0], layer_eps=[3.9],
        bc=(N, N, N, N, N, D), centre=(1.9, 2.0, 2.1), R=0.75, n=10, win_hi_z=2.55),
}


def _structure(c):
    hi = [4.0, 4.0, c.get("win_hi_z", 4.0)]
    return W.make_structure(c["cond"], c["nets"], c["diel"], c["diel_eps"], c["layer_z0"], c["layer_eps"],
                            [0.0, 0.0, 0.0], hi, c["bc"])


def _pin(st, centre, R, n, uncut=False):
    """The expanded cube's chain from the structure (float32 inputs as stored).
    uncut: links into absorbing nodes keep their full length (a planted
    mistake, for the sharpness check)."""
    c = np.asarray(centre, dtype=np.float64)
    h = 2 * R / n
    lo = c - R
    cond = st.cond.astype(np.float64)
    diel = st.diel.astype(np.float64)
    wlo, whi = st.win_lo.astype(np.float64), st.win_hi.astype(np.float64)
    z0 = st.layer_z0.astype(np.float64)
    codes = np.zeros((n, n, n))
    for k in range(n):
        for j in range(n):
            for i in range(n):
                p = lo + (np.array([i, j, k]) + 0.5) * h
                eps = None
                for b in range(st.n_diel - 1, -1, -1):
                    if np.all(p >= diel[b, :3]) and np.all(p < diel[b, 3:]):
                        eps = st.diel_eps[b]
                        break
                if eps is None:
                    eps = st.layer_eps[int(np.sum(p[2] >= z0[1:]))]
                codes[k, j, i] = np.rint(np.float64(eps) * 65536.0)

    def pos(i, j, k):
        return lo + np.array([i, j, k], dtype=np.float64) * h

    def grounded(x, a):
        return (st.bc[2 * a] == D and x[a] <= wlo[a]) or (st.bc[2 * a + 1] == D and x[a] >= whi[a])

    def node_net(i, j, k):
        x = pos(i, j, k)
        if any(grounded(x, a) for a in range(3)):
            return st.n_nets
        for b in range(st.n_cond):
            if np.all(x >= cond[b, :3]) and np.all(x <= cond[b, 3:]):
                return int(st.cond_net[b])
        return -1

    def cut_theta(i, j, k, d):
        a, up = d // 2, d % 2 == 1
        x = pos(i, j, k)
        th = []
        if up and st.bc[2 * a + 1] == D and x[a] + h >= whi[a]:
            th.append((whi[a] - x[a]) / h)
        if not up and st.bc[2 * a] == D and x[a] - h <= wlo[a]:
            th.append((x[a] - wlo[a]) / h)
        q = x.copy()
        q[a] += h if up else -h
        for b in range(st.n_cond):
            o = [e for e in range(3) if e != a]
            if not all(cond[b, e] <= x[e] <= cond[b, 3 + e] for e in o):
                continue
            if up and x[a] < cond[b, a] <= q[a]:
                th.append((cond[b, a] - x[a]) / h)
            if not up and q[a] <= cond[b, 3 + a] < x[a]:
                th.append((x[a] - cond[b, 3 + a]) / h)
        assert th, "link into an absorbing node meets no object"
        return min(th)

    return pins.expanded_cube_chain(codes, node_net, (lambda i, j, k, d: 1.0) if uncut else cut_theta)


@pytest.mark.parametrize("name", list(CASES))
def test_microwalk_e_walks_follow_absorbing_chain(oracle_lib, name):
    c = CASES[name]
    st = _structure(c)
    n, R = c["n"], c["R"]
    P, absorbed, etau = _pin(st, c["centre"], R, n)
    assert P.sum() + sum(absorbed.values()) == pytest.approx(1.0, abs=1e-12)
    # the case exercises absorption inside the cube by every kind of object
    assert set(absorbed) == set(range(st.n_nets + 1)) and min(absorbed.values()) > 0.01
    walks = 200000
    hits, nets, steps = oracle_lib.microwalk_e_cube(st, c["centre"], R, n, walks, seed=11, c1=3)
    M = n - 1
    cat = np.where(hits >= 0, hits, 6 * M * M + nets)
    counts = np.bincount(cat, minlength=6 * M * M + st.n_nets + 1)
    probs = np.concatenate([P, [absorbed[a] for a in range(st.n_nets + 1)]])
    p, stat, dof = pins.chi_square_p(counts, probs)
    print(name, "absorbed", absorbed, "chi2", stat, dof, "p", p, "E(tau)", etau, steps.mean())
    assert p > 1e-4
    se = steps.std() / np.sqrt(walks)
    assert abs(steps.mean() - etau) < 4 * se


def test_microwalk_e_pin_detects_a_wrong_theta(oracle_lib):
    """The pin is sharp enough to see a plausible mistake: the chain built
    with uncut links (theta = 1, the links of plain MicroWalk) is rejected by
    the oracle's walks."""
    c = CASES["face_and_conductor"]
    st = _structure(c)
    n, R = c["n"], c["R"]
    Pu, au, _ = _pin(st, c["centre"], R, n, uncut=True)
    hits, nets, _ = oracle_lib.microwalk_e_cube(st, c["centre"], R, n, 200000, seed=11, c1=3)
    M = n - 1
    cat = np.where(hits >= 0, hits, 6 * M * M + nets)
    counts = np.bincount(cat, minlength=6 * M * M + st.n_nets + 1)
    probs_u = np.concatenate([Pu, [au[a] for a in range(st.n_nets + 1)]])
    assert pins.chi_square_p(counts, probs_u)[0] < 1e-6
