"""Strong ROM-port constraint (SRPC) formulation, FP64 (Section 3.2: eqs. port_xp, port_g,
rom_port_matrix, rom_port_compatibility, rom_strong_constraint, gamma_map_port,
dd_lspg_NLP_rom_port; Section 5.2: eq. autoencoder_architecture_port; Section 7.6: the port
latent-size rule).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Every port j (a group of interface DoFs shared by the same set of subdomains P(j)) has one
decoder g_j^p of its own, acting on n_j^p port latents.  Subdomain i keeps its own copy of
the latents of every port it touches (Q(i) = the ports j with i in P(j)); its reduced
interface vector is the concatenation of those copies, in ascending port order, so
n_i^Gamma = sum_{j in Q(i)} n_j^p, and Phat_i^j picks port j's block.  The interface decoder
is implied by the port decoders (eq. gamma_map_port):

    g_i^Gamma(xhat_i^Gamma) = sum_{j in Q(i)} (P_i^j)^T g_j^p(Phat_i^j xhat_i^Gamma),

with P_i^j the rows of port j's DoFs inside x_i^Gamma.  The copies are tied together by the
linear constraint sum_i Ahat_i xhat_i^Gamma = 0 (eq. rom_strong_constraint): for every port
and every pair of consecutive carriers i_t < i_{t+1}, one row per port latent component
reading xhat_{i_t} - xhat_{i_{t+1}} = 0 (readings: rows ordered port-major, then carrier pair,
then component; +1 on the lower subdomain index, as for the FOM-port rows).  Its Jacobian
E_i = [0, Ahat_i] is constant.

Port latent sizes follow n_j^p = max(min(N_j^p - 1, n~), 1) for a requested n~.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from .autoencoder import Decoder, decode, decode_jacobian
from .ddmaps import DDMaps


def port_latent_size(N_p: int, n_tilde: int) -> int:
    """n_j^p = max(min(N_j^p - 1, n~), 1) (Section 7.6)."""
    return max(min(int(N_p) - 1, int(n_tilde)), 1)


@dataclass
class PortMaps:
    """Ports of a DD map and the SRPC bookkeeping per subdomain."""
    ports: list          # [(carriers (sorted subdomain ids), global DoFs ascending)]
    n_p: list            # latent size per port
    Q: list              # per subdomain: ascending port indices j with i in P(j)
    rows: list           # per subdomain: {j: positions of port j's DoFs inside x_i^Gamma}  (P_i^j)
    lat_off: list        # per subdomain: {j: offset of port j's latent copy inside xhat_i^Gamma}  (Phat_i^j)
    n_ga: list           # per subdomain: n_i^Gamma
    A_hat: list          # per subdomain: Ahat_i in {-1, 0, 1}^{n_A x n_i^Gamma} (dense)
    n_A: int


def build_port_maps(dd: DDMaps, n_p: list) -> PortMaps:
    ports = dd.ports
    if len(n_p) != len(ports):
        raise ValueError("one latent size per port")
    n_sub = dd.n_sub
    Q = [[] for _ in range(n_sub)]
    for j, (car, _) in enumerate(ports):
        for i in car:
            Q[i].append(j)
    rows, lat_off, n_ga = [], [], []
    for i, sd in enumerate(dd.subdomains):
        pos = {int(d): p for p, d in enumerate(sd.gamma)}
        r, o, off = {}, {}, 0
        for j in Q[i]:
            r[j] = np.array([pos[int(d)] for d in ports[j][1]], dtype=np.int64)
            o[j] = off
            off += n_p[j]
        rows.append(r)
        lat_off.append(o)
        n_ga.append(off)
    n_A = sum((len(car) - 1) * n_p[j] for j, (car, _) in enumerate(ports))
    A_hat = [np.zeros((n_A, n_ga[i])) for i in range(n_sub)]
    row = 0
    for j, (car, _) in enumerate(ports):
        for t in range(len(car) - 1):
            lo, hi = car[t], car[t + 1]
            for k in range(n_p[j]):
                A_hat[lo][row, lat_off[lo][j] + k] = 1.0
                A_hat[hi][row, lat_off[hi][j] + k] = -1.0
                row += 1
    return PortMaps(ports, list(n_p), Q, rows, lat_off, n_ga, A_hat, n_A)


class PortInterfaceDecoder:
    """g_i^Gamma of eq. gamma_map_port for one subdomain: a sum of its ports' decoders, each
    reading its own block of the subdomain's reduced interface vector."""

    def __init__(self, N_ga: int, parts: list):
        # parts: [(port decoder g_j^p, rows P_i^j inside x_i^Gamma, latent offset, latent size)]
        self.N_ga = int(N_ga)
        self.parts = parts
        self.n = sum(p[3] for p in parts)

    @property
    def N(self):
        return self.N_ga

    def decode(self, xhat: np.ndarray) -> np.ndarray:
        out = np.zeros(self.N_ga)
        for dec, rows, off, n in self.parts:
            out[rows] += decode(dec, xhat[off:off + n])
        return out

    def decode_jacobian(self, xhat: np.ndarray):
        out = np.zeros(self.N_ga)
        J = np.zeros((self.N_ga, self.n))
        for dec, rows, off, n in self.parts:
            g, Jp = decode_jacobian(dec, xhat[off:off + n])
            out[rows] += g
            J[np.ix_(rows, np.arange(off, off + n))] += Jp
        return out, J


def interface_decoders(dd: DDMaps, pm: PortMaps, port_decoders: list) -> list:
    out = []
    for i, sd in enumerate(dd.subdomains):
        parts = [(port_decoders[j], pm.rows[i][j], pm.lat_off[i][j], pm.n_p[j]) for j in pm.Q[i]]
        out.append(PortInterfaceDecoder(len(sd.gamma), parts))
    return out


def cover_ports(dd: DDMaps, hr_nodes: list) -> list:
    """Sampled nodes per subdomain, completed so that every port of the subdomain enters its
    hyper-reduced residual (reading; the paper does not discuss it): a port whose DoFs no
    sampled 5-point stencil reads leaves that port's latent copy without any effect on the
    subdomain's objective, its Gauss-Newton block singular, and Lemma 1 void.  For each such
    port the lowest owned node whose stencil reads one of the port's nodes is added."""
    g = dd.grid
    out = []
    for i, sd in enumerate(dd.subdomains):
        nodes = set(int(q) for q in hr_nodes[i])
        own = set(int(q) for q in sd.own_nodes)

        def stencil(p):
            j, ii = divmod(p, g.nx)
            st = [p]
            if ii > 0:
                st.append(p - 1)
            if ii < g.nx - 1:
                st.append(p + 1)
            if j > 0:
                st.append(p - g.nx)
            if j < g.ny - 1:
                st.append(p + g.nx)
            return st

        for car, dofs in dd.ports:
            if i not in car:
                continue
            pnodes = set(int(d) % g.n_nodes for d in dofs)
            if any(q in pnodes for p in nodes for q in stencil(p)):
                continue
            cand = sorted(p for p in own if any(q in pnodes for q in stencil(p)))
            nodes.add(cand[0])
        out.append(np.array(sorted(nodes), dtype=np.int64))
    return out
