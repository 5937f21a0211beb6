// Host-side construction of the device model: algebraic DD maps (Section 2), ports and
// compatibility matrices A_i, C A_i, interior decoder subnets (Section 5.4), stencil
// gather tables for the HR residual and the DD FOM residual, and the upload of all pools.
#include <algorithm>
#include <cstring>
#include <map>
#include <numeric>
#include <sstream>

#include "internal.h"

namespace ddrom {

static constexpr int RING = DEC_RING_WIDE;    // widest hidden-unit window the decode kernel takes
static constexpr int DEC_ROWS = 48;      // default max output rows per decode work item
static constexpr int DEC_STAGE = 15360;  // max bytes of FP32 weights staged in LDS per decode work item
static constexpr int RES_NODES = 24;     // default sampled nodes per residual work item
static constexpr int CON_ROWS = 8;       // constraint rows per constraint work item
static constexpr int CON_OROWS = 256;    // default interface rows per constraint work item

template <typename T>
static int upload(T** dst, const std::vector<T>& src) {
    size_t bytes = std::max<size_t>(1, src.size()) * sizeof(T);
    if (hipMalloc((void**)dst, bytes) != hipSuccess) {
        set_error("hipMalloc failed while uploading the model");
        return DDROM_ENOMEM;
    }
    if (!src.empty() && hipMemcpy(*dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice) != hipSuccess) {
        set_error("hipMemcpy failed while uploading the model");
        return DDROM_EHIP;
    }
    return 0;
}

struct HostDecoder {
    std::vector<double> W1, b1, W2, xref;   // packed subnet
    std::vector<int2> band;
    int rows = 0, hid = 0;
    int win = 0;        // widest hidden-unit window of a row
};

// Subnet of eq. subnet for the output rows `rows` (ascending) of one decoder.
// Dense output layer (every hidden unit feeds every row): one band per row covering all w
// hidden units, values in band slot 0 ([rows][3][w]).
static int make_dense_rows(const ddrom_decoder_desc& d, const std::vector<int>& rows, HostDecoder& out) {
    const int N = d.N, n = d.n, w = d.w;
    out.win = w;
    if (w > RING) {
        set_error("dense decoder wider than the kernel's hidden-unit ring (w must be <= 56)");
        return DDROM_EINVAL;
    }
    out.rows = (int)rows.size();
    out.hid = rows.empty() ? 0 : w;
    out.W1.assign(d.W1, d.W1 + (size_t)out.hid * n);
    out.b1.assign(d.b1, d.b1 + out.hid);
    out.band.assign(rows.size() * 3, int2{0, 0});
    out.W2.assign(rows.size() * 3 * (size_t)w, 0.0);
    out.xref.resize(rows.size());
    for (size_t q = 0; q < rows.size(); ++q) {
        const int r = rows[q];
        if (r < 0 || r >= N) {
            set_error("subnet row out of range");
            return DDROM_EINVAL;
        }
        out.xref[q] = d.x_ref[r];
        for (int t = 0; t < w; ++t) out.W2[q * 3 * w + t] = d.W2[(size_t)r * w + t];
        out.band[q * 3] = int2{0, w};
    }
    return 0;
}

static int make_subnet(const ddrom_decoder_desc& d, const std::vector<int>& rows, HostDecoder& out) {
    if (d.dense) return make_dense_rows(d, rows, out);
    const int N = d.N, n = d.n, w = d.w, b = d.b, s = d.s;
    std::vector<int> cmap(w, -1);
    for (int r : rows)
        for (int k = 0; k < 3; ++k)
            for (int t = 0; t < b; ++t) {
                long long c = (long long)r * s + (long long)(k - 1) * b * s + t;
                if (c >= 0 && c < w) cmap[c] = 1;
            }
    int hid = 0;
    std::vector<int> hidden;
    for (int c = 0; c < w; ++c)
        if (cmap[c] >= 0) {
            cmap[c] = hid++;
            hidden.push_back(c);
        }
    out.rows = (int)rows.size();
    out.hid = hid;
    out.W1.resize((size_t)hid * n);
    out.b1.resize(hid);
    for (int h = 0; h < hid; ++h) {
        for (int k = 0; k < n; ++k) out.W1[(size_t)h * n + k] = d.W1[(size_t)hidden[h] * n + k];
        out.b1[h] = d.b1[hidden[h]];
    }
    out.band.assign((size_t)rows.size() * 3, int2{0, 0});
    out.W2.assign((size_t)rows.size() * 3 * b, 0.0);
    out.xref.resize(rows.size());
    for (size_t q = 0; q < rows.size(); ++q) {
        int r = rows[q];
        if (r < 0 || r >= N) {
            set_error("subnet row out of range");
            return DDROM_EINVAL;
        }
        out.xref[q] = d.x_ref[r];
        int lo = 1 << 30, hi = -1;
        for (int k = 0; k < 3; ++k) {
            int t0 = -1, t1 = -1;
            for (int t = 0; t < b; ++t) {
                long long c = (long long)r * s + (long long)(k - 1) * b * s + t;
                if (c >= 0 && c < w) {
                    if (t0 < 0) t0 = t;
                    t1 = t;
                }
            }
            if (t0 < 0) continue;
            int c0 = r * s + (k - 1) * b * s + t0;
            int len = t1 - t0 + 1;
            int cs = cmap[c0];
            for (int t = 0; t < len; ++t) {
                if (cmap[c0 + t] != cs + t) {
                    set_error("internal: band not contiguous in the compressed hidden index");
                    return DDROM_EINVAL;
                }
                out.W2[(q * 3 + k) * b + t] = d.W2[((size_t)r * 3 + k) * b + t0 + t];
            }
            out.band[q * 3 + k] = int2{cs, len};
            lo = std::min(lo, cs);
            hi = std::max(hi, cs + len);
        }
        if (hi >= 0) out.win = std::max(out.win, hi - lo);
        if (hi >= 0 && hi - lo > RING) {
            set_error("decoder mask window wider than the kernel's hidden-unit ring (2*b*s + b must be <= 56)");
            return DDROM_EINVAL;
        }
    }
    return 0;
}

// Interface decoder of eq. gamma_map_port for one subdomain, assembled from the decoders of the
// ports it carries (block form of eq. interface_decoder_rom_port_blocks): the hidden units are the
// ports' hidden units, port by port in ascending port order; a hidden unit's W1~ row holds its port
// decoder's row in the columns of that port's latent copy (offset lat_off[a] inside xhat_i^Gamma)
// and zeros elsewhere; output row r (an interface state of the subdomain) takes the three bands
// of its port decoder's row for the same state, shifted to the port's hidden units.
static int make_port_interface(const ddrom_decoder_desc* pd, const std::vector<int>& Q,
                               const std::vector<int>& lat_off, int n_ga, const std::vector<int>& ifn_sd,
                               const std::vector<int>& port_of, const std::vector<int>& port_pos,
                               const std::vector<std::vector<int>>& port_nodes, int bmax, HostDecoder& out) {
    std::vector<int> hoff(Q.size()), qidx(port_nodes.size(), -1);
    int hid = 0;
    for (size_t a = 0; a < Q.size(); ++a) {
        hoff[a] = hid;
        hid += pd[Q[a]].w;
        qidx[Q[a]] = (int)a;
    }
    const int nif = (int)ifn_sd.size(), N = 2 * nif;
    out.rows = N;
    out.hid = hid;
    out.W1.assign((size_t)hid * n_ga, 0.0);
    out.b1.assign(hid, 0.0);
    for (size_t a = 0; a < Q.size(); ++a) {
        const ddrom_decoder_desc& e = pd[Q[a]];
        for (int c = 0; c < e.w; ++c) {
            for (int k = 0; k < e.n; ++k) out.W1[(size_t)(hoff[a] + c) * n_ga + lat_off[a] + k] = e.W1[(size_t)c * e.n + k];
            out.b1[hoff[a] + c] = e.b1[c];
        }
    }
    out.band.assign((size_t)N * 3, int2{0, 0});
    out.W2.assign((size_t)N * 3 * bmax, 0.0);
    out.xref.resize(N);
    for (int r = 0; r < N; ++r) {
        const int f = r / nif, q = ifn_sd[r % nif];
        const int j = port_of[q], a = qidx[j];
        if (j < 0 || a < 0) {
            set_error("internal: interface node outside the subdomain's ports");
            return DDROM_EINVAL;
        }
        const ddrom_decoder_desc& e = pd[j];
        const int p = port_pos[q] + f * (int)port_nodes[j].size();
        out.xref[r] = e.x_ref[p];
        int lo = 1 << 30, hi = -1;
        for (int k = 0; k < 3; ++k) {
            int t0 = -1, t1 = -1;
            for (int t = 0; t < e.b; ++t) {
                const long long c = (long long)p * e.s + (long long)(k - 1) * e.b * e.s + t;
                if (c >= 0 && c < e.w) {
                    if (t0 < 0) t0 = t;
                    t1 = t;
                }
            }
            if (t0 < 0) continue;
            const int c0 = p * e.s + (k - 1) * e.b * e.s + t0, len = t1 - t0 + 1;
            for (int t = 0; t < len; ++t) out.W2[((size_t)r * 3 + k) * bmax + t] = e.W2[((size_t)p * 3 + k) * e.b + t0 + t];
            out.band[(size_t)r * 3 + k] = int2{hoff[a] + c0, len};
            lo = std::min(lo, hoff[a] + c0);
            hi = std::max(hi, hoff[a] + c0 + len);
        }
        if (hi >= 0) out.win = std::max(out.win, hi - lo);
        if (hi >= 0 && hi - lo > RING) {
            set_error("port decoder mask window wider than the kernel's hidden-unit ring (2*b*s + b must be <= 56)");
            return DDROM_EINVAL;
        }
    }
    return 0;
}

int build_model(const ddrom_model_desc* d, ddrom_model* m) {
    if (!d || d->nx <= 0 || d->ny <= 0 || d->nsx <= 0 || d->nsy <= 0 || d->nx % d->nsx || d->ny % d->nsy) {
        set_error("grid must be positive and split evenly by nsx x nsy");
        return DDROM_EINVAL;
    }
    if (d->activation < 0 || d->activation > 2 || d->nu <= 0 || d->ly <= 0) {
        set_error("bad activation, viscosity or domain height");
        return DDROM_EINVAL;
    }
    const int nx = d->nx, ny = d->ny, nsx = d->nsx, nsy = d->nsy, n_sub = nsx * nsy;
    const int n_nodes = nx * ny, bx = nx / nsx, by = ny / nsy;
    m->nx = nx; m->ny = ny; m->nsx = nsx; m->nsy = nsy; m->n_sub = n_sub;
    m->act = d->activation; m->nu = d->nu; m->ly = d->ly;
    m->srpc = d->n_ports > 0 ? 1 : 0;
    m->act_ga = m->srpc ? d->port_activation : d->activation;
    if (m->srpc && (d->port_activation < 0 || d->port_activation > 2 || !d->dec_port)) {
        set_error("strong ROM-port constraint: bad port activation or no port decoders");
        return DDROM_EINVAL;
    }
    m->hx = 2.0 / (nx + 1); m->hy = d->ly / (ny + 1);
    m->N_x = 2 * n_nodes;
    m->n_C = d->n_C;
    m->tile_dec_rows = d->tile[0] > 0 ? d->tile[0] : DEC_ROWS;
    m->tile_res_nodes = d->tile[1] > 0 ? d->tile[1] : RES_NODES;
    m->tile_con_orows = d->tile[2] > 0 ? d->tile[2] : CON_OROWS;
    if (m->tile_dec_rows > 64 || m->tile_res_nodes < 4 || m->tile_con_orows < 4) {
        set_error("work-item shapes: decoder rows 1..64, residual nodes >= 4, constraint rows >= 4");
        return DDROM_EINVAL;
    }

    // ---- DD maps: owned, own-interface, halo, interior and interface nodes ----
    std::vector<int> owner(n_nodes);
    for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i) owner[j * nx + i] = (j / by) * nsx + (i / bx);
    std::vector<std::vector<int>> own(n_sub), intn(n_sub), ifn(n_sub);
    std::vector<std::vector<int>> halo(n_sub);
    for (int q = 0; q < n_nodes; ++q) own[owner[q]].push_back(q);
    std::vector<char> flag(n_nodes, 0);
    auto neighbours = [&](int q, int* out) {
        int j = q / nx, i = q % nx, c = 0;
        if (i > 0) out[c++] = q - 1;
        if (i < nx - 1) out[c++] = q + 1;
        if (j > 0) out[c++] = q - nx;
        if (j < ny - 1) out[c++] = q + nx;
        return c;
    };
    for (int sd = 0; sd < n_sub; ++sd) {
        std::vector<int> oif, hal;
        for (int q : own[sd]) {
            int nb[4], c = neighbours(q, nb), foreign = 0;
            for (int t = 0; t < c; ++t)
                if (owner[nb[t]] != sd) {
                    foreign = 1;
                    hal.push_back(nb[t]);
                }
            if (foreign) oif.push_back(q);
        }
        std::sort(hal.begin(), hal.end());
        hal.erase(std::unique(hal.begin(), hal.end()), hal.end());
        std::vector<char> oflag(n_nodes, 0);
        for (int q : oif) oflag[q] = 1;
        for (int q : own[sd])
            if (!oflag[q]) intn[sd].push_back(q);
        std::vector<int> all(oif);
        all.insert(all.end(), hal.begin(), hal.end());
        std::sort(all.begin(), all.end());
        ifn[sd] = all;
    }
    // ---- ports: groups of interface nodes carried by the same subdomains, numbered by their
    //      lowest node (every interface node has at least two carriers) ----
    std::vector<std::vector<int>> carriers(n_nodes);
    for (int sd = 0; sd < n_sub; ++sd)
        for (int q : ifn[sd]) carriers[q].push_back(sd);   // sd ascending by construction
    std::vector<int> port_of(n_nodes, -1), port_pos(n_nodes, -1);
    std::vector<std::vector<int>> port_nodes, port_car;
    std::vector<std::vector<int>> Qp(n_sub), lat_off(n_sub);
    std::vector<int> n_ga_srpc(n_sub, 0);
    int port_bmax = 1;
    if (m->srpc) {
        std::map<std::vector<int>, int> idx;
        for (int q = 0; q < n_nodes; ++q) {
            if (carriers[q].size() < 2) continue;
            auto it = idx.find(carriers[q]);
            int j;
            if (it == idx.end()) {
                j = (int)port_nodes.size();
                idx[carriers[q]] = j;
                port_nodes.push_back({});
                port_car.push_back(carriers[q]);
            } else {
                j = it->second;
            }
            port_of[q] = j;
            port_pos[q] = (int)port_nodes[j].size();
            port_nodes[j].push_back(q);
        }
        if ((int)port_nodes.size() != d->n_ports) {
            std::ostringstream os;
            os << "the split has " << port_nodes.size() << " ports, the descriptor " << d->n_ports;
            set_error(os.str());
            return DDROM_ESHAPE;
        }
        for (int j = 0; j < d->n_ports; ++j) {
            const ddrom_decoder_desc& e = d->dec_port[j];
            if (e.N != 2 * (int)port_nodes[j].size() || e.dense || e.n <= 0 || e.b <= 0 || e.s <= 0 || e.w != e.N * e.s || !e.W1 ||
                !e.b1 || !e.W2 || !e.x_ref) {
                std::ostringstream os;
                os << "port " << j << ": decoder needs N = " << 2 * port_nodes[j].size()
                   << " states, n, b, s > 0, w = N*s and all weight pointers";
                set_error(os.str());
                return DDROM_EINVAL;
            }
            port_bmax = std::max(port_bmax, e.b);
            for (int sd : port_car[j]) {
                Qp[sd].push_back(j);
                lat_off[sd].push_back(n_ga_srpc[sd]);
                n_ga_srpc[sd] += e.n;
            }
        }
        m->n_ports = d->n_ports;
    }

    m->n_om.resize(n_sub); m->n_ga.resize(n_sub); m->N_om.resize(n_sub); m->N_ga.resize(n_sub);
    m->xoff.resize(n_sub); m->n_own.resize(n_sub); m->nb.resize(n_sub); m->hid_om.resize(n_sub);
    m->state_off.resize(n_sub); m->res_off.resize(n_sub);
    int nD = 0;
    long long so = 0, ro = 0;
    for (int sd = 0; sd < n_sub; ++sd) {
        const ddrom_decoder_desc& a = d->dec_om[sd];
        ddrom_decoder_desc gport{};             // SRPC: the interface size only (weights come from ports)
        gport.N = 2 * (int)ifn[sd].size();
        const ddrom_decoder_desc& g = m->srpc ? gport : d->dec_ga[sd];
        m->N_om[sd] = 2 * (int)intn[sd].size();
        m->N_ga[sd] = 2 * (int)ifn[sd].size();
        m->n_own[sd] = (int)own[sd].size();
        if (a.N != m->N_om[sd] || g.N != m->N_ga[sd]) {
            std::ostringstream os;
            os << "subdomain " << sd << ": decoder sizes (" << a.N << ", " << g.N << ") do not match the DD split ("
               << m->N_om[sd] << ", " << m->N_ga[sd] << ")";
            set_error(os.str());
            return DDROM_ESHAPE;
        }
        for (const ddrom_decoder_desc* e : {&a, &g}) {
            if (e == &gport) continue;
            const bool shape_ok = e->dense ? (e->w > 0 && e->w <= RING) : (e->b > 0 && e->s > 0 && e->w == e->N * e->s);
            if (e->N > 0 && (e->n <= 0 || !shape_ok || !e->W1 || !e->b1 || !e->W2 || !e->x_ref)) {
                set_error("decoder descriptor: need n > 0, b, s > 0 and w = N*s (or dense with 0 < w <= 56) and all "
                          "weight pointers");
                return DDROM_EINVAL;
            }
            if (e->n > 24) {
                set_error("latent sizes above 24 are not supported");
                return DDROM_EINVAL;
            }
        }
        m->n_om[sd] = a.n;
        m->n_ga[sd] = m->srpc ? n_ga_srpc[sd] : (g.N > 0 ? g.n : 0);
        if (m->n_om[sd] + m->n_ga[sd] > 24 || m->n_ga[sd] > 12 || (m->n_om[sd] + m->n_ga[sd] > 20 && m->n_ga[sd] > 8)) {
            set_error("latent sizes beyond the KKT kernel's shapes (n_i^Omega + n_i^Gamma <= 20 with n_i^Gamma <= 12, "
                      "or <= 24 with n_i^Gamma <= 8)");
            return DDROM_EINVAL;
        }
        m->xoff[sd] = nD;
        nD += m->n_om[sd] + m->n_ga[sd];
        m->state_off[sd] = so;
        so += m->N_om[sd] + m->N_ga[sd];
        m->res_off[sd] = ro;
        ro += 2 * m->n_own[sd];
    }
    m->n_D = nD;
    m->n_state = (int)so;
    m->nmax = 0; m->mmax = 0; m->NNmax = 0;
    for (int sd = 0; sd < n_sub; ++sd) {
        m->nmax = std::max(m->nmax, m->n_om[sd] + m->n_ga[sd]);
        m->mmax = std::max(m->mmax, m->n_ga[sd]);
    }
    m->NNmax = m->nmax;
    if (m->srpc) {
        int nA = 0;
        for (int j = 0; j < m->n_ports; ++j) nA += ((int)port_car[j].size() - 1) * d->dec_port[j].n;
        m->n_C = nA;
    }
    if (m->n_C > 256) {
        set_error("n_C above 256 is not supported by the KKT kernel");
        return DDROM_EINVAL;
    }

    // ---- compatibility rows of the FOM ports, C A_i (weak constraint) or Ahat_i (strong) ----
    int n_A = 0;
    for (int q = 0; q < n_nodes; ++q)
        if (carriers[q].size() > 1) n_A += 2 * ((int)carriers[q].size() - 1);
    m->N_A = n_A;
    if (d->N_A != n_A) {
        std::ostringstream os;
        os << "C has " << d->N_A << " columns but the split has N_A = " << n_A << " compatibility conditions";
        set_error(os.str());
        return DDROM_ESHAPE;
    }
    if (!m->srpc && m->n_C > 0 && !d->C) {
        set_error("C is NULL");
        return DDROM_EINVAL;
    }
    auto pos_in = [](const std::vector<int>& v, int q) {
        return (int)(std::lower_bound(v.begin(), v.end(), q) - v.begin());
    };
    std::vector<std::vector<double>> CA(n_sub);
    for (int sd = 0; sd < n_sub; ++sd) CA[sd].assign(m->srpc ? 0 : (size_t)m->n_C * m->N_ga[sd], 0.0);
    std::vector<double> Ahat;      // SRPC: per subdomain [n_C][mmax]
    if (m->srpc) {
        const int mg = std::max(1, m->mmax);
        Ahat.assign((size_t)n_sub * m->n_C * mg, 0.0);
        int row = 0;
        for (int j = 0; j < m->n_ports; ++j) {
            const std::vector<int>& car = port_car[j];
            for (size_t t = 0; t + 1 < car.size(); ++t)
                for (int k = 0; k < d->dec_port[j].n; ++k, ++row) {
                    for (int side = 0; side < 2; ++side) {
                        const int sd = car[t + side];
                        const size_t a = std::find(Qp[sd].begin(), Qp[sd].end(), j) - Qp[sd].begin();
                        Ahat[((size_t)sd * m->n_C + row) * mg + lat_off[sd][a] + k] = side == 0 ? 1.0 : -1.0;
                    }
                }
        }
    }
    if (!m->srpc) {
        // rows ordered by global DoF: u-DoFs (node ascending) then v-DoFs
        int row = 0;
        for (int f = 0; f < 2; ++f)
            for (int q = 0; q < n_nodes; ++q) {
                const std::vector<int>& car = carriers[q];
                for (size_t t = 0; t + 1 < car.size(); ++t, ++row) {
                    int lo = car[t], hi = car[t + 1];
                    int plo = pos_in(ifn[lo], q) + f * (int)ifn[lo].size();
                    int phi = pos_in(ifn[hi], q) + f * (int)ifn[hi].size();
                    for (int j = 0; j < m->n_C; ++j) {
                        double c = d->C[(size_t)j * n_A + row];
                        CA[lo][(size_t)j * m->N_ga[lo] + plo] += c;
                        CA[hi][(size_t)j * m->N_ga[hi] + phi] -= c;
                    }
                }
            }
    }

    // ---- HR stencils, interior subnet rows, boundary points ----
    std::map<long long, int> bc_index;
    std::vector<double> bc_xy;
    std::vector<int> bc_field;
    auto bc_slot = [&](int I, int J, int field) {
        long long key = ((long long)I << 32) | ((long long)J << 1) | field;
        auto it = bc_index.find(key);
        if (it != bc_index.end()) return it->second;
        int k = (int)bc_field.size();
        bc_index[key] = k;
        bc_xy.push_back(-1.0 + I * m->hx);
        bc_xy.push_back(J * m->hy);
        bc_field.push_back(field);
        return k;
    };
    std::vector<int> gather;
    std::vector<std::vector<int>> gath_sd(n_sub);
    m->subnet_rows.resize(n_sub);
    for (int sd = 0; sd < n_sub; ++sd) {
        int cnt = d->hr_count ? d->hr_count[sd] : 0;
        if (cnt <= 0 || !d->hr_nodes || !d->hr_nodes[sd]) {
            set_error("every subdomain needs at least one HR node");
            return DDROM_EINVAL;
        }
        const int* hn = d->hr_nodes[sd];
        for (int k = 0; k < cnt; ++k) {
            if (hn[k] < 0 || hn[k] >= n_nodes || owner[hn[k]] != sd || (k > 0 && hn[k] <= hn[k - 1])) {
                set_error("HR nodes must be owned by their subdomain, ascending and unique");
                return DDROM_EINVAL;
            }
        }
        m->nb[sd] = cnt;
        const int nint = (int)intn[sd].size(), nif = (int)ifn[sd].size();
        std::vector<char> isint(n_nodes, 0);
        for (int q : intn[sd]) isint[q] = 1;
        std::vector<int> raw((size_t)cnt * N_SLOTS);
        std::vector<int> rows;
        for (int k = 0; k < cnt; ++k) {
            int q = hn[k], j = q / nx, i = q % nx;
            const int di[5] = {0, -1, 1, 0, 0}, dj[5] = {0, 0, 0, -1, 1};
            for (int t = 0; t < 5; ++t) {
                int ii = i + di[t], jj = j + dj[t];
                int cu, cv;
                if (ii < 0 || ii >= nx || jj < 0 || jj >= ny) {
                    cu = src_code(SRC_BOUND, bc_slot(ii + 1, jj + 1, 0));
                    cv = src_code(SRC_BOUND, bc_slot(ii + 1, jj + 1, 1));
                } else {
                    int r = jj * nx + ii;
                    if (owner[r] == sd && isint[r]) {
                        int p = pos_in(intn[sd], r);
                        cu = src_code(SRC_OMEGA, p);
                        cv = src_code(SRC_OMEGA, p + nint);
                        rows.push_back(p);
                        rows.push_back(p + nint);
                    } else {
                        int p = pos_in(ifn[sd], r);
                        cu = src_code(SRC_GAMMA, p);
                        cv = src_code(SRC_GAMMA, p + nif);
                    }
                }
                raw[(size_t)k * N_SLOTS + t] = cu;
                raw[(size_t)k * N_SLOTS + 5 + t] = cv;
            }
        }
        std::sort(rows.begin(), rows.end());
        rows.erase(std::unique(rows.begin(), rows.end()), rows.end());
        for (int& c : raw)
            if (src_kind(c) == SRC_OMEGA) c = src_code(SRC_OMEGA, pos_in(rows, src_index(c)));
        m->subnet_rows[sd] = rows;
        gath_sd[sd] = raw;
    }
    m->n_bc = (int)bc_field.size();

    // ---- decoders: interior subnets and full interface decoders (solver rounds, value and
    //      Jacobian rows), then full interior and interface decoders (values only, for the
    //      decoded subdomain states after a solve) ----
    std::vector<double> W1, b1, W2, xref;
    int maxwin = 0;
    std::vector<int2> bands;
    m->segs_h.assign(4 * n_sub, DecSeg{});
    m->band_nnz.assign(4 * n_sub, 0);
    long long out_rows = 0;
    for (int part = 0; part < 4; ++part)
        for (int sd = 0; sd < n_sub; ++sd) {
            const bool interior = part == 0 || part == 2;
            const bool ported = m->srpc && !interior;
            ddrom_decoder_desc pdesc{};
            pdesc.N = m->N_ga[sd];
            const ddrom_decoder_desc& dd = interior ? d->dec_om[sd] : (ported ? pdesc : d->dec_ga[sd]);
            DecSeg& sg = m->segs_h[part * n_sub + sd];
            sg.sd = sd;
            sg.n = interior ? m->n_om[sd] : m->n_ga[sd];
            sg.xoff = m->xoff[sd] + (interior ? 0 : m->n_om[sd]);
            sg.bmax = dd.N > 0 ? (ported ? port_bmax : (dd.dense ? dd.w : dd.b)) : 1;
            if (dd.N == 0) {
                sg.rows = 0; sg.hid = 0;
                sg.w1 = (long long)W1.size(); sg.b1 = (long long)b1.size(); sg.band = (long long)bands.size();
                sg.w2 = (long long)W2.size(); sg.xref = (long long)xref.size();
                sg.out = part < 2 ? out_rows : m->state_off[sd] + (part == 3 ? m->N_om[sd] : 0);
                continue;
            }
            std::vector<int> rows;
            if (part == 0) rows = m->subnet_rows[sd];
            else {
                rows.resize(dd.N);
                std::iota(rows.begin(), rows.end(), 0);
            }
            HostDecoder hd;
            int rc = ported ? make_port_interface(d->dec_port, Qp[sd], lat_off[sd], m->n_ga[sd], ifn[sd], port_of,
                                                  port_pos, port_nodes, port_bmax, hd)
                            : make_subnet(dd, rows, hd);
            if (rc) return rc;
            maxwin = std::max(maxwin, hd.win);
            sg.rows = hd.rows;
            sg.hid = hd.hid;
            sg.w1 = (long long)W1.size(); W1.insert(W1.end(), hd.W1.begin(), hd.W1.end());
            sg.b1 = (long long)b1.size(); b1.insert(b1.end(), hd.b1.begin(), hd.b1.end());
            sg.band = (long long)bands.size(); bands.insert(bands.end(), hd.band.begin(), hd.band.end());
            sg.w2 = (long long)W2.size(); W2.insert(W2.end(), hd.W2.begin(), hd.W2.end());
            sg.xref = (long long)xref.size(); xref.insert(xref.end(), hd.xref.begin(), hd.xref.end());
            if (part < 2) {
                sg.out = out_rows;
                out_rows += (long long)hd.rows * (1 + sg.n);
            } else {
                sg.out = m->state_off[sd] + (part == 3 ? m->N_om[sd] : 0);   // row of the state buffer
            }
            {
                long long nnz = 0;
                for (const int2& q : hd.band) nnz += q.y;
                m->band_nnz[part * n_sub + sd] = nnz;
            }
            if (part == 0) m->hid_om[sd] = hd.hid;
        }
    m->dec_rows = std::max<long long>(1, out_rows);
    m->ring = maxwin <= DEC_RING ? DEC_RING : DEC_RING_WIDE;
    // One work-item plan serves both precisions: the FP32 item (four waves, or two with the
    // Swish pair of rings) and the FP64 item (one wave, weights twice as wide) must both fit in
    // 64 KiB beside their rings.
    const int rk_max = (m->act == DDROM_ACT_SWISH || m->act_ga == DDROM_ACT_SWISH) ? 2 : 1;
    const int stage_budget = std::min({DEC_STAGE, 65536 - 128 - m->ring * 1024,
                                       (65536 - 128 - m->ring * 512 * rk_max) / 2});
    // Decode work items: runs of consecutive kept rows whose staged weights (W1~ rows and
    // biases of the hidden units they read, their W2~ values, x_ref, band descriptors) fit
    // in stage_budget bytes of FP32.
    m->seg_chunk0.assign(4 * n_sub, 0);
    m->seg_chunk1.assign(4 * n_sub, 0);
    m->seg_stage_f32.assign(4 * n_sub, 0);
    m->seg_stage_f64.assign(4 * n_sub, 0);
    for (int sgi = 0; sgi < 4 * n_sub; ++sgi) {
        m->seg_chunk0[sgi] = (int)m->chunks_h.size();
        const DecSeg& sg = m->segs_h[sgi];
        const int2* bd = bands.data() + sg.band;
        auto row_lo = [&](int r) {
            int lo = 1 << 30;
            for (int k = 0; k < 3; ++k)
                if (bd[r * 3 + k].y > 0) lo = std::min(lo, bd[r * 3 + k].x);
            return lo;
        };
        auto row_hi = [&](int r) {
            int hi = 0;
            for (int k = 0; k < 3; ++k)
                if (bd[r * 3 + k].y > 0) hi = std::max(hi, bd[r * 3 + k].x + bd[r * 3 + k].y);
            return hi;
        };
        int r = 0;
        while (r < sg.rows) {
            // The span is the union of the rows' windows (near the first rows a clipped band -1
            // can start below the first row's lowest band).  The kernel's ring holds the units
            // [vlo, vhi) with vhi - vlo <= m->ring; a row that would need a wider valid range starts
            // a new work item.
            int lo = row_lo(r), hi = row_hi(r), e = r + 1;
            int vlo = lo, vhi = hi;
            while (e < sg.rows && e - r < m->tile_dec_rows) {
                const int rl = row_lo(e), rh = row_hi(e);
                int nvlo = vlo, nvhi = vhi;
                if (rl >= nvhi || rh <= nvlo) nvlo = nvhi = rl;
                nvlo = std::min(nvlo, rl);
                nvhi = std::max(nvhi, rh);
                if (nvhi - rl > m->ring) break;
                nvlo = std::max(nvlo, nvhi - m->ring);
                int nlo = std::min(lo, rl), nhi = std::max(hi, rh);
                long long bytes = 4LL * ((long long)(nhi - nlo) * (sg.n + 1) + (long long)(e + 1 - r) * (3 * sg.bmax + 1)) +
                                  24LL * (e + 1 - r);
                if (bytes > stage_budget) break;
                lo = nlo;
                hi = nhi;
                vlo = nvlo;
                vhi = nvhi;
                ++e;
            }
            m->chunks_h.push_back(DecChunk{sgi, r, e, lo, hi, {0, 0, 0}});
            m->seg_stage_f32[sgi] = std::max<long long>(m->seg_stage_f32[sgi], (long long)dec_lds(hi - lo, e - r, sg.n, sg.bmax, 4, 0, 1, m->ring).ring);
            m->seg_stage_f64[sgi] = std::max<long long>(m->seg_stage_f64[sgi], (long long)dec_lds(hi - lo, e - r, sg.n, sg.bmax, 8, 0, 1, m->ring).ring);
            r = e;
        }
        m->seg_chunk1[sgi] = (int)m->chunks_h.size();
    }

    // ---- decoder launch plans: per family, segments of equal latent size (ascending) become
    //      one contiguous run of work items, each segment's items still contiguous ----
    {
        std::vector<DecChunk> sorted;
        sorted.reserve(m->chunks_h.size());
        std::vector<int> c0(4 * n_sub, 0), c1(4 * n_sub, 0);
        for (int f = 0; f < 4; ++f) {
            std::vector<int> order(n_sub);
            for (int sd = 0; sd < n_sub; ++sd) order[sd] = f * n_sub + sd;
            std::stable_sort(order.begin(), order.end(),
                             [&](int a, int b) { return m->segs_h[a].n < m->segs_h[b].n; });
            for (size_t k = 0; k < order.size();) {
                size_t e = k + 1;
                while (e < order.size() && m->segs_h[order[e]].n == m->segs_h[order[k]].n) ++e;
                ddrom_model::DecPlan pl{(int)sorted.size(), 0, m->segs_h[order[k]].n, 0, 0};
                for (size_t q = k; q < e; ++q) {
                    const int g = order[q];
                    c0[g] = (int)sorted.size();
                    for (int c = m->seg_chunk0[g]; c < m->seg_chunk1[g]; ++c) sorted.push_back(m->chunks_h[c]);
                    c1[g] = (int)sorted.size();
                    pl.stage_f32 = std::max(pl.stage_f32, m->seg_stage_f32[g]);
                    pl.stage_f64 = std::max(pl.stage_f64, m->seg_stage_f64[g]);
                }
                pl.c1 = (int)sorted.size();
                if (pl.c1 > pl.c0) m->dec_plan[f].push_back(pl);
                k = e;
            }
        }
        m->chunks_h.swap(sorted);
        m->seg_chunk0.swap(c0);
        m->seg_chunk1.swap(c1);
    }

    // ---- residual work items and GN partial slots ----
    m->rsegs_h.resize(n_sub);
    int slot = 0;
    m->estride = 0;
    for (int sd = 0; sd < n_sub; ++sd) {
        ResSeg& rs = m->rsegs_h[sd];
        rs.n_om = m->n_om[sd];
        rs.n_ga = m->n_ga[sd];
        rs.seg_om = sd;
        rs.seg_ga = n_sub + sd;
        rs.gather = (long long)gather.size();
        gather.insert(gather.end(), gath_sd[sd].begin(), gath_sd[sd].end());
        rs.slot0 = slot;
        for (int p = 0; p < m->nb[sd]; p += m->tile_res_nodes)
            m->rchunks_h.push_back(ResChunk{sd, p, std::min(m->nb[sd], p + m->tile_res_nodes), slot++});
        rs.slot1 = slot;
        int NN = rs.n_om + rs.n_ga;
        m->estride = std::max(m->estride, NN * (NN + 1) / 2 + NN + 1);
    }
    m->n_slots = slot;
    // residual launch plan: work items grouped by (n_i^Omega, n_i^Gamma); each item keeps its
    // partial slot, and the slots of a subdomain stay consecutive for the reduction
    {
        std::vector<int> order(n_sub);
        for (int sd = 0; sd < n_sub; ++sd) order[sd] = sd;
        auto cls = [&](int sd) { return std::make_pair(m->n_om[sd], m->n_ga[sd]); };
        std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return cls(a) < cls(b); });
        std::vector<ResChunk> sorted;
        sorted.reserve(m->rchunks_h.size());
        for (size_t k = 0; k < order.size();) {
            size_t e = k + 1;
            while (e < order.size() && cls(order[e]) == cls(order[k])) ++e;
            ddrom_model::ResPlan pl{(int)sorted.size(), 0, m->n_om[order[k]], m->n_ga[order[k]]};
            for (size_t q = k; q < e; ++q) {
                const ResSeg& rs = m->rsegs_h[order[q]];
                for (int sl = rs.slot0; sl < rs.slot1; ++sl) sorted.push_back(m->rchunks_h[sl]);
            }
            pl.c1 = (int)sorted.size();
            if (pl.c1 > pl.c0) m->res_plan.push_back(pl);
            k = e;
        }
        m->rchunks_h.swap(sorted);
    }

    // ---- gappy-POD hyper-reduction: stored rows, projection items, one GN slot per subdomain ----
    std::vector<double> gP;
    std::vector<int2> gitems;
    if (d->hr_modes) {
        if (!d->hr_gappy) {
            set_error("gappy POD: hr_gappy is NULL");
            return DDROM_EINVAL;
        }
        m->gappy = 1;
        m->gseg_h.resize(n_sub);
        long long ro = 0, yo = 0;
        for (int sd = 0; sd < n_sub; ++sd) {
            GappySeg& g = m->gseg_h[sd];
            g.nn = m->n_om[sd] + m->n_ga[sd];
            g.nb = m->nb[sd];
            g.rows = 2 * g.nb;
            g.modes = d->hr_modes[sd];
            if (g.modes < 1 || g.modes > g.rows || !d->hr_gappy[sd] || g.nn > 12) {
                set_error("gappy POD: need 1 <= hr_modes[i] <= 2 hr_count[i], the matrix, and n_i <= 12");
                return DDROM_EINVAL;
            }
            g.r_off = ro;
            g.y_off = yo;
            g.p_off = (long long)gP.size();
            ro += (long long)g.rows * (g.nn + 1);
            yo += (long long)g.modes * (g.nn + 1);
            gP.insert(gP.end(), d->hr_gappy[sd], d->hr_gappy[sd] + (size_t)g.modes * g.rows);
            for (int q = 0; q < g.modes; q += ddrom::kGappyModes) gitems.push_back(int2{sd, q});
            // the projected sums of a subdomain go to one partial slot
            m->rsegs_h[sd].slot0 = sd;
            m->rsegs_h[sd].slot1 = sd + 1;
        }
        m->n_slots = n_sub;
        m->g_rrows = ro;
        m->g_yrows = yo;
        m->n_gitems = (int)gitems.size();
    }

    // ---- constraint work items ----
    std::vector<ConChunk> cch;
    std::vector<double> CAflat;
    m->CA_off.resize(n_sub);
    m->ca_ld = (m->n_C + 7) / 8 * 8;
    std::vector<int> cchunk0(n_sub + 1, 0);
    int cpart = 0;
    for (int sd = 0; sd < n_sub; ++sd) {
        const int Ng = m->N_ga[sd];
        m->CA_off[sd] = (long long)CAflat.size();
        m->rsegs_h[sd].ca = m->CA_off[sd];
        m->rsegs_h[sd].n_rows_ga = Ng;
        // (C A_i)^T, rows of length ca_ld so that a work item's 8 multipliers are contiguous
        if (!m->srpc) {
            std::vector<double> t((size_t)Ng * m->ca_ld, 0.0);
            for (int j = 0; j < m->n_C; ++j)
                for (int o = 0; o < Ng; ++o) t[(size_t)o * m->ca_ld + j] = CA[sd][(size_t)j * Ng + o];
            CAflat.insert(CAflat.end(), t.begin(), t.end());
        }
        m->rsegs_h[sd].cpart0 = cpart;
        cchunk0[sd] = (int)cch.size();
        const int orows = m->tile_con_orows;
        if (m->srpc) {
            // the linear constraint's partials are formed per subdomain by their own kernel
            if (m->n_C > 0) ++cpart;
        } else if (Ng > 0 && m->n_C > 0)
            for (int o = 0; o < Ng; o += orows, ++cpart)
                for (int j = 0; j < m->n_C; j += CON_ROWS)
                    cch.push_back(ConChunk{sd, j, std::min(m->n_C, j + CON_ROWS), o, std::min(Ng, o + orows), cpart, {0, 0}});
        m->rsegs_h[sd].cpart1 = cpart;
    }
    cchunk0[n_sub] = (int)cch.size();
    m->n_cchunks = (int)cch.size();
    m->n_cparts = cpart;
    // constraint launch plan: work items grouped by n_i^Gamma
    {
        std::vector<int> order(n_sub);
        for (int sd = 0; sd < n_sub; ++sd) order[sd] = sd;
        std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return m->n_ga[a] < m->n_ga[b]; });
        std::vector<ConChunk> sorted;
        sorted.reserve(cch.size());
        for (size_t k = 0; k < order.size();) {
            size_t e = k + 1;
            while (e < order.size() && m->n_ga[order[e]] == m->n_ga[order[k]]) ++e;
            ddrom_model::ConPlan pl{(int)sorted.size(), 0, m->n_ga[order[k]]};
            for (size_t q = k; q < e; ++q)
                for (int c = cchunk0[order[q]]; c < cchunk0[order[q] + 1]; ++c) sorted.push_back(cch[c]);
            pl.c1 = (int)sorted.size();
            if (pl.c1 > pl.c0) m->con_plan.push_back(pl);
            k = e;
        }
        cch.swap(sorted);
    }

    // ---- DD FOM residual tables ----
    std::vector<int> fsrc;
    std::vector<long long> fmeta;
    std::vector<int> sd_of_row;
    int own_off = 0;
    for (int sd = 0; sd < n_sub; ++sd) {
        const int nint = (int)intn[sd].size(), nif = (int)ifn[sd].size();
        std::vector<char> isint(n_nodes, 0);
        for (int q : intn[sd]) isint[q] = 1;
        for (int q : own[sd]) {
            int j = q / nx, i = q % nx;
            const int di[5] = {0, -1, 1, 0, 0}, dj[5] = {0, 0, 0, -1, 1};
            for (int t = 0; t < 5; ++t) {
                int ii = i + di[t], jj = j + dj[t];
                int code;
                if (ii < 0 || ii >= nx || jj < 0 || jj >= ny) code = src_code(SRC_BOUND, ((ii + 1) << 14) | (jj + 1));
                else {
                    int r = jj * nx + ii;
                    if (owner[r] == sd && isint[r]) code = src_code(SRC_OMEGA, pos_in(intn[sd], r));
                    else code = src_code(SRC_GAMMA, pos_in(ifn[sd], r));
                }
                fsrc.push_back(code);
            }
            sd_of_row.push_back(sd);
        }
        fmeta.insert(fmeta.end(), {(long long)own_off, (long long)own[sd].size(), (long long)nint, (long long)nif,
                                   m->state_off[sd], m->res_off[sd]});
        own_off += (int)own[sd].size();
    }
    m->total_own = own_off;
    if (nx + 2 >= (1 << 14) || ny + 2 >= (1 << 14)) {
        set_error("grid too large for the boundary code packing");
        return DDROM_EINVAL;
    }

    // ---- global DoF of every row of the DD state [x_1^Omega; x_1^Gamma; ...] ----
    std::vector<int> state_dof((size_t)m->n_state);
    {
        const int nn = nx * ny;
        for (int sd = 0; sd < n_sub; ++sd) {
            const int nint = (int)intn[sd].size(), nif = (int)ifn[sd].size();
            long long o = m->state_off[sd];
            for (int f = 0; f < 2; ++f)
                for (int p = 0; p < nint; ++p) state_dof[o++] = intn[sd][p] + f * nn;
            for (int f = 0; f < 2; ++f)
                for (int p = 0; p < nif; ++p) state_dof[o++] = ifn[sd][p] + f * nn;
        }
    }

    // ---- upload ----
    std::vector<float> W1f(W1.begin(), W1.end()), b1f(b1.begin(), b1.end()), W2f(W2.begin(), W2.end()),
        xreff(xref.begin(), xref.end());
    int rc = 0;
    if ((rc = upload(&m->W1d, W1)) || (rc = upload(&m->b1d, b1)) || (rc = upload(&m->W2d, W2)) ||
        (rc = upload(&m->xrefd, xref)) || (rc = upload(&m->W1f, W1f)) || (rc = upload(&m->b1f, b1f)) ||
        (rc = upload(&m->W2f, W2f)) || (rc = upload(&m->xreff, xreff)) || (rc = upload(&m->bands, bands)) ||
        (rc = upload(&m->segs_d, m->segs_h)) || (rc = upload(&m->chunks_d, m->chunks_h)) ||
        (rc = upload(&m->gather_d, gather)) || (rc = upload(&m->rsegs_d, m->rsegs_h)) ||
        (rc = upload(&m->rchunks_d, m->rchunks_h)) || (rc = upload(&m->bc_xy_d, bc_xy)) ||
        (rc = upload(&m->bc_field_d, bc_field)) || (rc = upload(&m->CA_d, CAflat)) ||
        (rc = upload(&m->cchunks_d, cch)) || (rc = upload(&m->fom_src_d, fsrc)) ||
        (rc = upload(&m->fom_meta_d, fmeta)) || (rc = upload(&m->fom_sd_of_row_d, sd_of_row)) ||
        (rc = upload(&m->state_dof_d, state_dof)) || (rc = upload(&m->Ahat_d, Ahat)) ||
        (m->gappy && ((rc = upload(&m->gseg_d, m->gseg_h)) || (rc = upload(&m->gP_d, gP)) ||
                      (rc = upload(&m->gitems_d, gitems)))))
        return rc;
    return 0;
}

void free_model(ddrom_model* m) {
    void* ptrs[] = {m->W1f, m->b1f, m->W2f, m->xreff, m->W1d, m->b1d, m->W2d, m->xrefd, m->bands, m->segs_d,
                    m->chunks_d, m->gather_d, m->rsegs_d, m->rchunks_d, m->bc_xy_d, m->bc_field_d, m->CA_d,
                    m->cchunks_d, m->fom_src_d, m->fom_meta_d, m->fom_sd_of_row_d, m->state_dof_d, m->Ahat_d,
                    m->gseg_d, m->gP_d, m->gitems_d};
    for (void* p : ptrs)
        if (p) (void)hipFree(p);
}

}  // namespace ddrom
