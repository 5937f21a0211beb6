"""Algebraic domain decomposition of the Burgers FOM (Section 2).

For a uniform nsx x nsy block split of the interior node grid (subdomain index
i = sy*nsx + sx, x-fastest):

  * residual sampling P_i^r: the r_u and r_v rows of the nodes subdomain i owns;
  * interior states x_i^Omega: DoFs of owned nodes whose 5-point stencil stays inside
    subdomain i (they enter no other subdomain's residual);
  * interface states x_i^Gamma: DoFs of owned nodes with a stencil neighbour in another
    subdomain, plus the other subdomains' nodes that appear in stencils of owned nodes;
  * ports: interface DoFs grouped by the set of subdomains whose interface vectors
    contain them; each port j has |P(j)|-1 chained equality conditions per DoF;
  * A_i in {-1,0,1}^{N_A x N_i^Gamma} with sum_i A_i x_i^Gamma = 0.

Orderings (readings; the paper fixes none of them): every sampled vector lists global
DoF indices in ascending order (so u-DoFs precede v-DoFs).  Constraint rows are ordered
by the global DoF they duplicate, ascending; for a DoF shared by subdomains
i_1 < ... < i_k the rows t = 1..k-1 read x_{i_t} - x_{i_{t+1}} = 0 (+1 on the lower
subdomain index, -1 on the higher).  The feasible set does not depend on these choices.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp

from .burgers import Grid


@dataclass
class Subdomain:
    index: int
    own_nodes: np.ndarray        # global node ids (j*nx + i, 0-based interior nodes), ascending
    res_rows: np.ndarray         # P_i^r: global residual rows, ascending
    omega: np.ndarray            # P_i^Omega: global DoF indices, ascending
    gamma: np.ndarray            # P_i^Gamma: global DoF indices, ascending


@dataclass
class DDMaps:
    grid: Grid
    nsx: int
    nsy: int
    subdomains: list
    A: list                      # A_i as scipy.sparse csr, N_A x N_i^Gamma
    n_A: int
    ports: list                  # list of (tuple(sorted subdomain ids), np.array of global DoFs)

    @property
    def n_sub(self) -> int:
        return len(self.subdomains)


def node_owner(g: Grid, nsx: int, nsy: int) -> np.ndarray:
    """Owner subdomain of every interior node (node id = j*nx + i)."""
    if g.nx % nsx or g.ny % nsy:
        raise ValueError("grid must split evenly")
    bx, by = g.nx // nsx, g.ny // nsy
    i = np.arange(g.nx)
    j = np.arange(g.ny)
    own = (j[:, None] // by) * nsx + (i[None, :] // bx)
    return own.ravel()


def stencil_neighbours(g: Grid, node: int):
    """Interior 5-point neighbours (W, E, S, N) of a node; boundary nodes are omitted."""
    j, i = divmod(int(node), g.nx)
    out = []
    if i > 0:
        out.append(node - 1)
    if i < g.nx - 1:
        out.append(node + 1)
    if j > 0:
        out.append(node - g.nx)
    if j < g.ny - 1:
        out.append(node + g.nx)
    return out


def build_dd(g: Grid, nsx: int, nsy: int) -> DDMaps:
    owner = node_owner(g, nsx, nsy)
    n_nodes = g.n_nodes
    n_sub = nsx * nsy
    own_iface = [set() for _ in range(n_sub)]
    halo = [set() for _ in range(n_sub)]
    for node in range(n_nodes):
        o = owner[node]
        for nb in stencil_neighbours(g, node):
            if owner[nb] != o:
                own_iface[o].add(node)   # node's own residual needs a foreign state
                halo[o].add(nb)          # foreign state entering subdomain o's residual
    subs = []
    for s in range(n_sub):
        own = np.flatnonzero(owner == s)
        iface_nodes = np.array(sorted(own_iface[s] | halo[s]), dtype=np.int64)
        interior_nodes = np.array(sorted(set(own.tolist()) - own_iface[s]), dtype=np.int64)
        res_rows = np.concatenate([own, own + n_nodes])
        omega = np.concatenate([interior_nodes, interior_nodes + n_nodes])
        gamma = np.concatenate([iface_nodes, iface_nodes + n_nodes])
        subs.append(Subdomain(s, own, res_rows, omega, gamma))

    # Which subdomains carry each interface DoF.
    carriers: dict[int, list] = {}
    for s, sd in enumerate(subs):
        for d in sd.gamma:
            carriers.setdefault(int(d), []).append(s)
    ports: dict[tuple, list] = {}
    for d, lst in carriers.items():
        ports.setdefault(tuple(sorted(lst)), []).append(d)
    port_list = sorted(((k, np.array(sorted(v))) for k, v in ports.items()), key=lambda kv: (kv[1][0], kv[0]))

    pos = [{int(d): p for p, d in enumerate(sd.gamma)} for sd in subs]
    rows = [[] for _ in range(n_sub)]
    cols = [[] for _ in range(n_sub)]
    vals = [[] for _ in range(n_sub)]
    r = 0
    for d in sorted(carriers):
        lst = sorted(carriers[d])
        for t in range(len(lst) - 1):
            lo, hi = lst[t], lst[t + 1]
            rows[lo].append(r); cols[lo].append(pos[lo][d]); vals[lo].append(1.0)
            rows[hi].append(r); cols[hi].append(pos[hi][d]); vals[hi].append(-1.0)
            r += 1
    n_A = r
    A = [sp.csr_matrix((vals[s], (rows[s], cols[s])), shape=(n_A, len(subs[s].gamma))) for s in range(n_sub)]
    return DDMaps(g, nsx, nsy, subs, A, n_A, port_list)


def restrict(dd: DDMaps, x: np.ndarray):
    """(P_i^Omega x, P_i^Gamma x) for every subdomain."""
    return [(x[sd.omega], x[sd.gamma]) for sd in dd.subdomains]


def subdomain_residual(fom, dd: DDMaps, i: int, x_om: np.ndarray, x_ga: np.ndarray, mu):
    """r_i(x^Omega, x^Gamma) = P_i^r r((P_i^Omega)^T x^Omega + (P_i^Gamma)^T x^Gamma)
    (eq. subdomain_residual_def), with the Jacobian blocks w.r.t. x^Omega and x^Gamma."""
    sd = dd.subdomains[i]
    x = np.zeros(dd.grid.n_dof)
    x[sd.omega] = x_om
    x[sd.gamma] = x_ga
    r = fom.residual(x, mu)[sd.res_rows]
    return r


def subdomain_residual_jac(fom, dd: DDMaps, i: int, x_om, x_ga, mu):
    sd = dd.subdomains[i]
    x = np.zeros(dd.grid.n_dof)
    x[sd.omega] = x_om
    x[sd.gamma] = x_ga
    r = fom.residual(x, mu)[sd.res_rows]
    J = fom.jacobian(x, mu)[sd.res_rows]
    return r, J[:, sd.omega], J[:, sd.gamma]
