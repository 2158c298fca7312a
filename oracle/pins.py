"""Independent checks for the oracle (TEST INFRASTRUCTURE ONLY).

Library solves (scipy sparse LU) of the finite-difference systems of
Sec. III-A and III-B of Huang & Yu (arXiv 2507.09730), and closed-form
harmonic functions, used to pin the C++ oracle's MicroWalk (Alg. 3) and its
conjugate-gradient SGF solver to something other than themselves.
"""
import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

DIRS = np.array([[-1, 0, 0], [1, 0, 0], [0, -1, 0], [0, 1, 0], [0, 0, -1], [0, 0, 1]])


def vertex_boundary_nodes(n):
    """Coordinates (6 M^2 x 3) of the reachable boundary nodes of the vertex
    lattice in hit-index order f*M^2 + (b-1)*M + (a-1)."""
    M = n - 1
    out = np.zeros((6 * M * M, 3), dtype=np.int64)
    for f in range(6):
        ax, side = divmod(f, 2)
        o0 = 1 if ax == 0 else 0
        o1 = 1 if ax == 2 else 2
        for b in range(1, n):
            for a in range(1, n):
                h = f * M * M + (b - 1) * M + (a - 1)
                out[h, ax] = n if side else 0
                out[h, o0] = a
                out[h, o1] = b
    return out


def vertex_exit_distribution(links, n, src=None):
    """Absorbing-chain solve (Eq. 9 and Theorem 1 via Grinstead & Snell,
    Thm. 11.6 / 11.5) on the vertex lattice from the per-node link codes.

    links: (M^3, 6) codes, node order ((k-1)M+(j-1))M+(i-1).  Builds
    Q_II, Q_IB from p_d = g_d / sum(g) and solves (I - Q_II)^T x = e_src with
    a sparse LU.  Returns (P over 6 M^2 hit indices, E(tau))."""
    M = n - 1
    NI = M ** 3
    links = np.asarray(links, dtype=np.float64)
    p = links / links.sum(axis=1, keepdims=True)
    coords = np.stack(np.meshgrid(np.arange(1, n), np.arange(1, n), np.arange(1, n),
                                  indexing="ij"), axis=-1)
    # node index order: i fastest
    idx = lambda i, j, k: ((k - 1) * M + (j - 1)) * M + (i - 1)
    bnodes = vertex_boundary_nodes(n)
    bindex = {tuple(c): h for h, c in enumerate(bnodes)}
    rows, cols, vals = [], [], []
    brow, bcol, bval = [], [], []
    for k in range(1, n):
        for j in range(1, n):
            for i in range(1, n):
                v = idx(i, j, k)
                for d in range(6):
                    q = (i + DIRS[d, 0], j + DIRS[d, 1], k + DIRS[d, 2])
                    if min(q) == 0 or max(q) == n:
                        brow.append(v)
                        bcol.append(bindex[q])
                        bval.append(p[v, d])
                    else:
                        rows.append(v)
                        cols.append(idx(*q))
                        vals.append(p[v, d])
    Q = sp.csr_matrix((vals, (rows, cols)), shape=(NI, NI))
    QB = sp.csr_matrix((bval, (brow, bcol)), shape=(NI, 6 * M * M))
    A = (sp.identity(NI, format="csc") - Q.tocsc())
    if src is None:
        src = (n // 2,) * 3
    e = np.zeros(NI)
    e[idx(*src)] = 1.0
    x = spla.spsolve(A.T.tocsc(), e)  # row e_src^T (I - Q)^-1
    P = QB.T @ x
    return np.asarray(P).ravel(), float(x.sum())


def cell_exit_distribution(links, N, src=None):
    """Same solve on the cell-centred lattice of Sec. III-A (Eq. 6 codes),
    nodes (k*N+j)*N+i, hit index f*N^2 + b*N + a; src (i, j, k) defaults to
    the centre cell."""
    NI = N ** 3
    links = np.asarray(links, dtype=np.float64)
    p = links / links.sum(axis=1, keepdims=True)
    rows, cols, vals = [], [], []
    brow, bcol, bval = [], [], []
    for k in range(N):
        for j in range(N):
            for i in range(N):
                v = (k * N + j) * N + i
                for d in range(6):
                    q = [i + DIRS[d, 0], j + DIRS[d, 1], k + DIRS[d, 2]]
                    ax = d // 2
                    if q[ax] < 0 or q[ax] >= N:
                        side = 1 if q[ax] >= N else 0
                        a = q[1] if ax == 0 else q[0]
                        b = q[1] if ax == 2 else q[2]
                        brow.append(v)
                        bcol.append((2 * ax + side) * N * N + b * N + a)
                        bval.append(p[v, d])
                    else:
                        rows.append(v)
                        cols.append((q[2] * N + q[1]) * N + q[0])
                        vals.append(p[v, d])
    Q = sp.csr_matrix((vals, (rows, cols)), shape=(NI, NI))
    QB = sp.csr_matrix((bval, (brow, bcol)), shape=(NI, 6 * N * N))
    A = sp.identity(NI, format="csc") - Q.tocsc()
    if src is None:
        src = ((N - 1) // 2,) * 3
    e = np.zeros(NI)
    e[(src[2] * N + src[1]) * N + src[0]] = 1.0
    x = spla.spsolve(A.T.tocsc(), e)
    return np.asarray(QB.T @ x).ravel(), float(x.sum())


def chi_square_p(counts, probs, min_expected=5.0):
    """Pearson chi-square p-value of observed counts against probabilities,
    pooling bins with expected count below min_expected."""
    from scipy.stats import chi2
    counts = np.asarray(counts, dtype=np.float64)
    probs = np.asarray(probs, dtype=np.float64)
    n = counts.sum()
    exp = probs * n
    big = exp >= min_expected
    obs = list(counts[big])
    ex = list(exp[big])
    if (~big).any():
        obs.append(counts[~big].sum())
        ex.append(exp[~big].sum())
    obs, ex = np.array(obs), np.array(ex)
    keep = ex > 0
    stat = float(((obs[keep] - ex[keep]) ** 2 / ex[keep]).sum())
    dof = int(keep.sum()) - 1
    return float(chi2.sf(stat, dof)), stat, dof


def series_potential(eps_layers):
    """Node potentials of the 1-D series stack along an axis: constant flux
    eps_k * (phi_{k+1} - phi_k) / h across each cell layer k (interface
    condition of Eq. 4), phi_0 = 0.  Returns n+1 node potentials."""
    phi = [0.0]
    for e in eps_layers:
        phi.append(phi[-1] + 1.0 / float(e))
    return np.array(phi)


def vertex_links_from_codes(codes):
    """Link codes of every interior node of the vertex lattice from the cell
    codes (numpy, written independently of the C++ oracle): the link of
    direction d is the sum of the four cells that share its edge.  codes:
    (n, n, n) indexed [k, j, i].  Returns an (n-1)^3 x 6 array in node order
    ((k-1)M+(j-1))M+(i-1), directions -x,+x,-y,+y,-z,+z."""
    E = np.asarray(codes, dtype=np.int64)
    n = E.shape[0]
    M = n - 1
    out = np.zeros((M ** 3, 6), dtype=np.int64)
    for k in range(1, n):
        for j in range(1, n):
            for i in range(1, n):
                v = ((k - 1) * M + (j - 1)) * M + (i - 1)
                out[v, 0] = E[k - 1:k + 1, j - 1:j + 1, i - 1].sum()
                out[v, 1] = E[k - 1:k + 1, j - 1:j + 1, i].sum()
                out[v, 2] = E[k - 1:k + 1, j - 1, i - 1:i + 1].sum()
                out[v, 3] = E[k - 1:k + 1, j, i - 1:i + 1].sum()
                out[v, 4] = E[k - 1, j - 1:j + 1, i - 1:i + 1].sum()
                out[v, 5] = E[k, j - 1:j + 1, i - 1:i + 1].sum()
    return out


def expanded_cube_chain(codes, node_net, cut_theta):
    """Absorbing-chain solve of a MicroWalk-E cube (Sec. III-B with Theorem 1):
    the vertex lattice of Alg. 3 in which some interior nodes are absorbing
    (inside a conductor, or beyond a grounded face) and the links into them
    are shortened to the fraction theta of their length at which they meet
    the object, their code becoming rint(code / theta) (the Shortley-Weller
    form of a Dirichlet boundary between nodes).

    codes: (n, n, n) cell codes [k, j, i]; node_net(i, j, k): the absorbing net
    of an interior node or -1; cut_theta(i, j, k, d): theta of the link from
    free node (i, j, k) in direction d into an absorbing node.  Returns
    (P over the 6 M^2 boundary hit indices, {net: probability}, E(tau)) for
    walks from the centre node, by a sparse LU solve of (I - Q)^T x = e_c."""
    n = np.asarray(codes).shape[0]
    M = n - 1
    links = vertex_links_from_codes(codes)
    idx = lambda i, j, k: ((k - 1) * M + (j - 1)) * M + (i - 1)
    bnodes = vertex_boundary_nodes(n)
    bindex = {tuple(c): h for h, c in enumerate(bnodes)}
    free = {}
    nets = {}
    for k in range(1, n):
        for j in range(1, n):
            for i in range(1, n):
                a = node_net(i, j, k)
                if a < 0:
                    free[(i, j, k)] = len(free)
                else:
                    nets[(i, j, k)] = a
    labels = sorted(set(nets.values()))
    lab_index = {a: q for q, a in enumerate(labels)}
    NF = len(free)
    rows, cols, vals = [], [], []
    brow, bcol, bval = [], [], []
    arow, acol, aval = [], [], []
    for (i, j, k), v in free.items():
        g = links[idx(i, j, k)].astype(np.float64)
        for d in range(6):
            q = (i + DIRS[d, 0], j + DIRS[d, 1], k + DIRS[d, 2])
            if q in nets:
                th = max(cut_theta(i, j, k, d), 1.0 / 16.0)
                g[d] = np.rint(g[d] / th)
        p = g / g.sum()
        for d in range(6):
            q = (i + DIRS[d, 0], j + DIRS[d, 1], k + DIRS[d, 2])
            if min(q) == 0 or max(q) == n:
                brow.append(v)
                bcol.append(bindex[q])
                bval.append(p[d])
            elif q in nets:
                arow.append(v)
                acol.append(lab_index[nets[q]])
                aval.append(p[d])
            else:
                rows.append(v)
                cols.append(free[q])
                vals.append(p[d])
    Q = sp.csr_matrix((vals, (rows, cols)), shape=(NF, NF))
    QB = sp.csr_matrix((bval, (brow, bcol)), shape=(NF, 6 * M * M))
    QA = sp.csr_matrix((aval, (arow, acol)), shape=(NF, max(len(labels), 1)))
    A = sp.identity(NF, format="csc") - Q.tocsc()
    e = np.zeros(NF)
    e[free[(n // 2,) * 3]] = 1.0
    x = spla.spsolve(A.T.tocsc(), e)
    P = np.asarray(QB.T @ x).ravel()
    pa = np.asarray(QA.T @ x).ravel()
    return P, {a: float(pa[lab_index[a]]) for a in labels}, float(x.sum())
