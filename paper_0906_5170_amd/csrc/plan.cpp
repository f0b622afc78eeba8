// Host planning: walls, stress surface, interpolation, cosine basis,
// channel table, update coefficients and the time kernel.
#include "plan.hpp"

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdio>
#include <set>

namespace cf {

// E_a: half a cell along a.  H_a: half a cell along both other axes.
const int kOffset2[kNumComp][3] = {
    {1, 0, 0}, {0, 1, 0}, {0, 0, 1},   // Ex Ey Ez
    {0, 1, 1}, {1, 0, 1}, {1, 1, 0},   // Hx Hy Hz
};

static bool is_e(int comp) { return comp < 3; }

void pol_components(int pol, std::vector<int>& e, std::vector<int>& h) {
    e.clear();
    h.clear();
    if (pol == CF_POL_TM) {
        e = {CF_EZ};
        h = {CF_HX, CF_HY};
    } else if (pol == CF_POL_TE) {
        e = {CF_EX, CF_EY};
        h = {CF_HZ};
    } else {
        e = {CF_EX, CF_EY, CF_EZ};
        h = {CF_HX, CF_HY, CF_HZ};
    }
}

// Field block of a channel: TM (Ez, Hx, Hy), TE (Ex, Ey, Hz), 3D (Ex..Hz).
int comp_slot(int pol, int comp) {
    if (pol == CF_POL_TM) return comp == CF_EZ ? 0 : comp == CF_HX ? 1 : comp == CF_HY ? 2 : -1;
    if (pol == CF_POL_TE) return comp == CF_EX ? 0 : comp == CF_EY ? 1 : comp == CF_HZ ? 2 : -1;
    return comp;
}

int n_comp_for(int ndim) { return ndim == 2 ? 3 : 6; }

int n_comp(const Problem& p) { return p.bloch ? 12 : p.reduced() ? 6 : n_comp_for(p.grid.ndim); }

double order_courant(const Problem& p, double courant, int m) {
    return p.cyl && m >= 2 ? std::min(courant, 1.0 / (1.0 + m)) : courant;
}

// Same physical time t_end = n_steps courant / res for every order; the
// rounding is half-to-even (nearbyint in the default rounding mode).
int order_steps(const Problem& p, const cf_opts& o, int m) {
    if (!p.cyl) return o.n_steps;
    const double dx = 1.0 / p.grid.res;
    const double t_end = o.n_steps * o.courant * dx;
    return (int)std::nearbyint(t_end / (order_courant(p, o.courant, m) * dx));
}

int max_steps(const Problem& p, const cf_opts& o) {
    int t = o.n_steps;
    if (p.cyl)
        for (int m = 0; m <= p.m_max; ++m) t = std::max(t, order_steps(p, o, m));
    return t;
}

int harmonic_len(const Problem& p) {
    int lab = 0;
    for (auto& v : p.labels)
        for (int l : v) lab = std::max(lab, l + 1);
    if (p.reduced()) lab += (p.n_orders() - 1) * p.surf.n_harm;
    return lab;
}

static bool spans_periodic(const Problem& p, int a) {
    return p.grid.bc[a] == CF_BC_PERIODIC && p.surf.lo[a] == 0 && p.surf.hi[a] == p.grid.n[a];
}

// Points along one axis for a sample at doubled coordinate s2 and a
// component with doubled offset o2: one point (weight 1) when they coincide,
// else the two neighbours with weight 1/2.
static bool axis_points(int s2, int o2, int n, bool periodic, int* i, double* w, int* np) {
    int d = s2 - o2;
    if ((d % 2 + 2) % 2 == 0) {
        i[0] = d / 2;
        w[0] = 1.0;
        *np = 1;
    } else {
        i[0] = (d - 1) / 2;
        i[1] = (d + 1) / 2;
        w[0] = w[1] = 0.5;
        *np = 2;
    }
    for (int k = 0; k < *np; ++k) {
        if (periodic) {
            i[k] = ((i[k] % n) + n) % n;
        } else if (i[k] < 0 || i[k] >= n) {
            return false;
        }
    }
    return true;
}

static std::string make_gather(const Problem& p, int fi, int comp, Gather& g) {
    const Face& f = p.faces[fi];
    g.face = fi;
    g.comp = comp;
    g.nsamp = f.nsamp;
    g.P = 0;
    g.idx.clear();
    g.w.clear();
    for (int s = 0; s < f.nsamp; ++s) {
        int t[2] = {0, 0};
        if (f.ntang == 1) {
            t[0] = s;
        } else {
            t[0] = s / f.count[1];
            t[1] = s % f.count[1];
        }
        int pi[3][2];
        double pw[3][2];
        int pn[3];
        for (int ax = 0; ax < 3; ++ax) {
            if (ax >= p.grid.ndim) {
                pi[ax][0] = 0;
                pw[ax][0] = 1.0;
                pn[ax] = 1;
                continue;
            }
            int s2;
            if (ax == f.axis) {
                s2 = 2 * f.plane;
            } else {
                int k = (f.tang[0] == ax) ? 0 : 1;
                s2 = 2 * (f.start[k] + t[k]) + 1;
            }
            if (!axis_points(s2, kOffset2[comp][ax], p.grid.n[ax], p.grid.bc[ax] == CF_BC_PERIODIC,
                             pi[ax], pw[ax], &pn[ax]))
                return "stress surface stencil leaves the grid";
        }
        int count = 0;
        for (int a = 0; a < pn[0]; ++a)
            for (int b = 0; b < pn[1]; ++b)
                for (int c = 0; c < pn[2]; ++c) {
                    int64_t flat = ((int64_t)pi[2][c] * p.ny + pi[1][b]) * p.nx + pi[0][a];
                    g.idx.push_back((int32_t)flat);
                    g.w.push_back(pw[0][a] * pw[1][b] * pw[2][c]);
                    ++count;
                }
        if (s == 0) g.P = count;
        if (count != g.P) return "non-uniform interpolation stencil";
    }
    // adjoint (scatter) form, distinct points in ascending order
    std::map<int32_t, std::vector<std::pair<int32_t, double>>> by_point;
    for (int s = 0; s < g.nsamp; ++s)
        for (int q = 0; q < g.P; ++q) by_point[g.idx[s * g.P + q]].push_back({s, g.w[s * g.P + q]});
    g.uidx.clear();
    g.uoff.assign(1, 0);
    g.usamp.clear();
    g.uw.clear();
    for (auto& kv : by_point) {
        g.uidx.push_back(kv.first);
        for (auto& sw : kv.second) {
            g.usamp.push_back(sw.first);
            g.uw.push_back(sw.second);
        }
        g.uoff.push_back((int32_t)g.usamp.size());
    }
    return "";
}

// Cosine basis on N midpoints of a face of length L = N dx:
// f_0 = sqrt(1/L), f_n = sqrt(2/L) cos(n pi (i + 1/2) / N).
static std::vector<double> cosine_rows(int N, int nh, double dx) {
    int rows = std::min(nh, N);
    std::vector<double> b((size_t)rows * N);
    double L = N * dx;
    for (int n = 0; n < rows; ++n) {
        double c = std::sqrt((n == 0 ? 1.0 : 2.0) / L);
        for (int i = 0; i < N; ++i) b[(size_t)n * N + i] = c * std::cos(M_PI * n * (i + 0.5) / N);
    }
    return b;
}

static std::string surface_medium(Problem& p);
static std::string finish_cyl_surface(Problem& p, const cf_surface& s);

// ---- cylindrical surfaces --------------------------------------------------
//
// The (z, r) rectangle lo..hi in cells; r = y - 1/2 with y the grid's axis-1
// coordinate, so the doubled y of radius r is 2 r + 1.

// Points along one axis for doubled coordinate d2 and component offset o2;
// points at or beyond n on a non-periodic axis lie in or past the wall
// (field zero there) and are left out; false if a point falls below 0.
static bool cyl_axis_points(int d2, int o2, int n, bool periodic, std::vector<std::pair<int, double>>& out) {
    out.clear();
    const int d = d2 - o2;
    int pi[2];
    double pw[2];
    int np;
    if ((d % 2 + 2) % 2 == 0) {
        pi[0] = d / 2;
        pw[0] = 1.0;
        np = 1;
    } else {
        pi[0] = (d - 1) / 2;
        pi[1] = (d + 1) / 2;
        pw[0] = pw[1] = 0.5;
        np = 2;
    }
    for (int k = 0; k < np; ++k) {
        int i = pi[k];
        if (periodic) {
            i = ((i % n) + n) % n;
        } else if (i >= n) {
            continue;
        } else if (i < 0) {
            return false;
        }
        out.push_back({i, pw[k]});
    }
    return true;
}

static void cyl_faces(const Problem& p, const cf_surface& s, std::vector<Face>& faces) {
    const int nr = p.ny;
    const int z0 = s.lo[0], z1 = s.hi[0], r0 = s.lo[1], r1 = s.hi[1];
    const bool to_wall = r1 >= nr;
    std::vector<int> ys, xs;
    std::vector<double> wy, wx;
    for (int k = r0; k < (to_wall ? nr - 1 : r1); ++k) {
        ys.push_back(2 * k + 2);      // r = k + 1/2
        wy.push_back(1.0);
    }
    if (to_wall) {
        ys.push_back(2 * nr - 1);     // r = nr - 1: the half cell up to the wall
        wy.push_back(0.5);
    }
    for (int i = z0; i < z1; ++i) {
        xs.push_back(2 * i + 1);
        wx.push_back(1.0);
    }
    auto make = [&](int axis, int side, int plane2, const std::vector<int>& s2, const std::vector<double>& w) {
        Face f{};
        f.index = 2 * axis + (side > 0);
        f.axis = axis;
        f.side = side;
        f.plane = plane2 / 2;
        f.plane2 = plane2;
        f.ntang = 1;
        f.tang[0] = 1 - axis;
        f.start[0] = 0;
        f.count[0] = (int)s2.size();
        f.nsamp = (int)s2.size();
        f.samp2 = s2;
        f.qw = w;
        faces.push_back(f);
    };
    make(0, -1, 2 * z0, ys, wy);
    make(0, +1, 2 * z1, ys, wy);
    if (r0 > 0) make(1, -1, 2 * r0 + 1, xs, wx);
    if (!to_wall) make(1, +1, 2 * r1 + 1, xs, wx);
}

// Rows w_s f_n(s) of the first min(nh, N) members of the cosine basis made
// orthonormal under dx sum_s w_s f g (classical Gram-Schmidt in FP64, in
// order n = 0, 1, ...); cos(n pi pos / L) at the sample's position pos
// along the face (cumulative weights), L the face length in cells.
static std::vector<double> weighted_cosine_rows(const std::vector<double>& w, int nh, double dx) {
    const int N = (int)w.size();
    const int rows = std::min(nh, N);
    std::vector<double> pos(N);
    double L = 0;
    for (int i = 0; i < N; ++i) {
        pos[i] = L + 0.5 * w[i];
        L += w[i];
    }
    std::vector<std::vector<double>> f;
    for (int n = 0; n < rows; ++n) {
        std::vector<double> v(N);
        for (int i = 0; i < N; ++i) v[i] = std::cos(n * M_PI * pos[i] / L);
        for (const auto& u : f) {
            double dot = 0;
            for (int i = 0; i < N; ++i) dot += w[i] * u[i] * v[i];
            dot *= dx;
            for (int i = 0; i < N; ++i) v[i] -= dot * u[i];
        }
        double nn = 0;
        for (int i = 0; i < N; ++i) nn += w[i] * v[i] * v[i];
        nn = std::sqrt(dx * nn);
        for (int i = 0; i < N; ++i) v[i] /= nn;
        f.push_back(std::move(v));
    }
    std::vector<double> b((size_t)rows * N);
    for (int n = 0; n < rows; ++n)
        for (int i = 0; i < N; ++i) b[(size_t)n * N + i] = w[i] * f[n][i];
    return b;
}

// Gather of one component on a cylindrical face.  order_one: the axis rows
// of E_r and H_phi (Ey, Hz) read the next row (m = 1) instead of zero.
// Samples with fewer points are padded with zero-weight copies of their
// first point so every sample has the same point count.
static std::string make_gather_cyl(const Problem& p, int fi, int comp, bool order_one, Gather& g) {
    const Face& f = p.faces[fi];
    g.face = fi;
    g.comp = comp;
    g.nsamp = f.nsamp;
    std::vector<std::vector<std::pair<int32_t, double>>> pts(f.nsamp);
    std::vector<std::pair<int, double>> pz, pr;
    const bool per_z = p.grid.bc[0] == CF_BC_PERIODIC;
    const bool axis_copy = comp == CF_EY || comp == CF_HZ;
    int P = 0;
    for (int s = 0; s < f.nsamp; ++s) {
        const int zd = f.axis == 0 ? f.plane2 : f.samp2[s];
        const int rd = f.axis == 0 ? f.samp2[s] : f.plane2;
        if (!cyl_axis_points(zd, kOffset2[comp][0], p.nx, per_z, pz) ||
            !cyl_axis_points(rd, kOffset2[comp][1], p.ny, false, pr))
            return "stress surface stencil leaves the grid";
        for (auto& a : pz)
            for (auto& b : pr) {
                int j = b.first;
                double w = a.second * b.second;
                if (axis_copy && j == 0) {
                    if (order_one) j = 1;
                    else w = 0.0;
                }
                pts[s].push_back({(int32_t)((int64_t)j * p.nx + a.first), w});
            }
        if (pts[s].empty()) return "stress surface sample lies outside the grid";
        P = std::max(P, (int)pts[s].size());
    }
    g.P = P;
    g.idx.clear();
    g.w.clear();
    for (int s = 0; s < f.nsamp; ++s) {
        for (int q = 0; q < P; ++q) {
            const bool real = q < (int)pts[s].size();
            g.idx.push_back(real ? pts[s][q].first : pts[s][0].first);
            g.w.push_back(real ? pts[s][q].second : 0.0);
        }
    }
    std::map<int32_t, std::vector<std::pair<int32_t, double>>> by_point;
    for (int s = 0; s < g.nsamp; ++s)
        for (int q = 0; q < g.P; ++q)
            if (g.w[s * g.P + q] != 0.0) by_point[g.idx[s * g.P + q]].push_back({s, g.w[s * g.P + q]});
    g.uidx.clear();
    g.uoff.assign(1, 0);
    g.usamp.clear();
    g.uw.clear();
    for (auto& kv : by_point) {
        g.uidx.push_back(kv.first);
        for (auto& sw : kv.second) {
            g.usamp.push_back(sw.first);
            g.uw.push_back(sw.second);
        }
        g.uoff.push_back((int32_t)g.usamp.size());
    }
    return "";
}

std::string build_problem(const cf_grid& g, const cf_materials& m, const cf_surface& s,
                          Problem& p) {
    static std::atomic<uint64_t> next_uid{1};
    p.uid = next_uid.fetch_add(1);
    if (g.ndim != 2 && g.ndim != 3) return "ndim must be 2 or 3";
    for (int a = 0; a < 3; ++a)
        if (g.n[a] < 1) return "grid sizes must be positive";
    if (g.ndim == 2 && g.n[2] != 1) return "2D grids need n[2] == 1";
    if (!(g.res > 0)) return "res must be positive";
    int64_t ncell = (int64_t)g.n[0] * g.n[1] * g.n[2];
    if (ncell >= (int64_t)1 << 31) return "grid too large for 32-bit cell indices";
    for (int a = 0; a < g.ndim; ++a) {
        if (g.bc[a] < CF_BC_PEC || g.bc[a] > CF_BC_PML) return "unknown boundary";
        if (g.bc[a] == CF_BC_PML && (g.pml_cells[a] < 1 || 2 * g.pml_cells[a] >= g.n[a]))
            return "PML thickness out of range";
    }
    if (g.coord != CF_COORD_CARTESIAN && g.coord != CF_COORD_CYLINDRICAL && g.coord != CF_COORD_KZ)
        return "unknown coordinate system";
    if (g.coord == CF_COORD_KZ) {
        if (g.ndim != 2) return "k_z problems are 2D grids";
        if (s.n_kz < 1 || s.n_kz > 33 || !s.kz || !s.kz_weight) return "k_z problems need 1..33 wavevectors";
        for (int q = 0; q < s.n_kz; ++q)
            if (!std::isfinite(s.kz[q]) || !std::isfinite(s.kz_weight[q])) return "k_z points must be finite";
    }
    if (g.coord == CF_COORD_CYLINDRICAL) {
        if (g.ndim != 2) return "cylindrical problems are 2D (r, z) grids";
        if (g.bc[1] != CF_BC_PEC) return "cylindrical problems need a PEC tube wall (bc[1])";
        if (s.m_max < 0 || s.m_max > 32) return "m_max must be in 0..32";
    }
    if (m.n_materials < 1 || m.n_materials > 254 || !m.eps || !m.mu) return "bad material table";
    p.grid = g;
    p.cyl = g.coord == CF_COORD_CYLINDRICAL;
    p.kz = g.coord == CF_COORD_KZ;
    p.m_max = p.cyl ? s.m_max : 0;
    p.kzs.clear();
    p.kz_w.clear();
    p.kxs.clear();
    p.bloch = false;
    if (p.kz) {
        p.kzs.assign(s.kz, s.kz + s.n_kz);
        p.kz_w.assign(s.kz_weight, s.kz_weight + s.n_kz);
        p.kxs.assign(s.n_kz, 0.0);
        if (s.kx)
            for (int q = 0; q < s.n_kz; ++q) {
                if (!std::isfinite(s.kx[q])) return "k_x points must be finite";
                p.kxs[q] = s.kx[q];
                p.bloch = p.bloch || s.kx[q] != 0.0;
            }
        if (p.bloch && g.bc[0] != CF_BC_PERIODIC) return "Bloch-periodic x needs a periodic x axis";
    }
    if (g.ndim == 2) {
        p.grid.bc[2] = CF_BC_PERIODIC;
        p.grid.pml_cells[2] = 0;
    }
    p.nx = g.n[0];
    p.ny = g.n[1];
    p.nz = g.n[2];
    p.ncell = ncell;
    p.nmat = m.n_materials;
    p.eps.assign(m.eps, m.eps + m.n_materials);
    p.mu.assign(m.mu, m.mu + m.n_materials);
    for (int i = 0; i < p.nmat; ++i) {
        bool pec = std::isinf(p.eps[i]) && p.eps[i] < 0;
        bool pmc = std::isinf(p.mu[i]) && p.mu[i] < 0;
        if (!pec && !(p.eps[i] > 0 && std::isfinite(p.eps[i]))) return "eps must be > 0 or -inf";
        if (!pmc && !(p.mu[i] > 0 && std::isfinite(p.mu[i]))) return "mu must be > 0 or -inf";
    }
    std::vector<char> used(p.nmat, 0);
    for (int c = 0; c < kNumComp; ++c) {
        if (m.comp_id[c]) {
            p.ids[c].assign(m.comp_id[c], m.comp_id[c] + ncell);
            for (uint8_t v : p.ids[c]) {
                if (v >= p.nmat) return "material id out of range";
                used[v] = 1;
            }
        } else {
            p.ids[c].assign(ncell, 0);
            used[0] = 1;
        }
    }
    // Lorentz terms of dispersive materials
    p.n_lor = 0;
    p.lor_de.clear();
    p.lor_w0.clear();
    p.dispersive = false;
    if (m.n_lorentz < 0 || m.n_lorentz > 4) return "n_lorentz must be in 0..4";
    if (m.n_lorentz > 0 && m.lorentz_deps && m.lorentz_w0) {
        p.n_lor = m.n_lorentz;
        const size_t n = (size_t)p.nmat * p.n_lor;
        p.lor_de.assign(m.lorentz_deps, m.lorentz_deps + n);
        p.lor_w0.assign(m.lorentz_w0, m.lorentz_w0 + n);
        for (size_t k = 0; k < n; ++k)
            if (!std::isfinite(p.lor_de[k]) || !std::isfinite(p.lor_w0[k]) || !(p.lor_w0[k] > 0 || p.lor_de[k] == 0))
                return "Lorentz terms need finite d_eps and w0 > 0";
    }
    // Appendix A.2's kernel assumes perfect conductors in vacuum: note
    // whether every material the grid uses is vacuum or a perfect conductor
    p.vacuum_conductors = true;
    for (int i = 0; i < p.nmat; ++i) {
        if (!used[i]) continue;
        const bool conductor = (std::isinf(p.eps[i]) && p.eps[i] < 0) || (std::isinf(p.mu[i]) && p.mu[i] < 0);
        const bool terms = !(std::isinf(p.eps[i]) && p.eps[i] < 0) && p.has_terms(i);
        p.dispersive = p.dispersive || terms;
        if (!conductor && (terms || !(p.eps[i] == 1.0 && p.mu[i] == 1.0))) p.vacuum_conductors = false;
    }
    // E components lying on a PEC(-backed) wall: integer coordinate 0 along
    // a non-periodic axis.
    for (int c = 0; c < 3; ++c)
        for (int a = 0; a < p.grid.ndim; ++a) {
            if (p.grid.bc[a] == CF_BC_PERIODIC || kOffset2[c][a] != 0) continue;
            for (int k = 0; k < p.nz; ++k)
                for (int j = 0; j < p.ny; ++j)
                    for (int i = 0; i < p.nx; ++i) {
                        int coord = a == 0 ? i : a == 1 ? j : k;
                        if (coord == 0) p.ids[c][((int64_t)k * p.ny + j) * p.nx + i] = kWallId;
                    }
        }
    // stress surface
    p.surf = s;
    p.surf.kz = nullptr;          // copied into kzs / kz_w / kxs above
    p.surf.kz_weight = nullptr;
    p.surf.kx = nullptr;
    if (s.force_axis < 0 || s.force_axis >= g.ndim) return "force_axis out of range";
    if (s.n_harm < 1) return "n_harm must be >= 1";
    p.faces.clear();
    if (p.cyl) {
        if (s.force_axis != 0) return "cylindrical problems take the axial force (force_axis 0)";
        if (s.lo[0] >= s.hi[0] || s.lo[1] >= s.hi[1]) return "surface box is empty";
        if (s.lo[1] < 0 || s.hi[1] > p.ny) return "stress surface leaves the grid radially";
        cyl_faces(p, s, p.faces);
        return finish_cyl_surface(p, s);
    }
    for (int a = 0; a < g.ndim; ++a) {
        if (s.lo[a] >= s.hi[a]) return "surface box is empty";
        if (spans_periodic(p, a)) continue;
        Face f{};
        f.axis = a;
        f.ntang = 0;
        f.nsamp = 1;
        for (int b = 0; b < g.ndim; ++b) {
            if (b == a) continue;
            f.tang[f.ntang] = b;
            f.start[f.ntang] = s.lo[b];
            f.count[f.ntang] = s.hi[b] - s.lo[b];
            f.nsamp *= f.count[f.ntang];
            ++f.ntang;
        }
        for (int side : {-1, +1}) {
            f.side = side;
            f.plane = side < 0 ? s.lo[a] : s.hi[a];
            f.index = 2 * a + (side > 0);
            p.faces.push_back(f);
        }
    }
    if (p.faces.empty()) return "surface has no faces";
    double dx = 1.0 / g.res;
    p.basis.clear();
    p.labels.clear();
    p.nrows.clear();
    for (const Face& f : p.faces) {
        if (f.ntang == 1) {
            auto b = cosine_rows(f.count[0], s.n_harm, dx);
            int rows = (int)(b.size() / f.count[0]);
            std::vector<int> lab(rows);
            for (int r = 0; r < rows; ++r) lab[r] = r;
            p.basis.push_back(b);
            p.labels.push_back(lab);
            p.nrows.push_back(rows);
        } else {
            auto bu = cosine_rows(f.count[0], s.n_harm, dx);
            auto bv = cosine_rows(f.count[1], s.n_harm, dx);
            int ru = (int)(bu.size() / f.count[0]), rv = (int)(bv.size() / f.count[1]);
            std::vector<double> b((size_t)ru * rv * f.nsamp);
            std::vector<int> lab;
            for (int mm = 0; mm < ru; ++mm)
                for (int nn = 0; nn < rv; ++nn) {
                    size_t row = (size_t)mm * rv + nn;
                    for (int i0 = 0; i0 < f.count[0]; ++i0)
                        for (int i1 = 0; i1 < f.count[1]; ++i1)
                            b[row * f.nsamp + (size_t)i0 * f.count[1] + i1] =
                                bu[(size_t)mm * f.count[0] + i0] * bv[(size_t)nn * f.count[1] + i1];
                    lab.push_back(mm * s.n_harm + nn);
                }
            p.basis.push_back(b);
            p.labels.push_back(lab);
            p.nrows.push_back(ru * rv);
        }
    }
    // interpolation tables for every (face, component)
    p.gathers.clear();
    p.gather_of.clear();
    for (int fi = 0; fi < (int)p.faces.size(); ++fi)
        for (int c = 0; c < kNumComp; ++c) {
            Gather gt;
            std::string err = make_gather(p, fi, c, gt);
            if (!err.empty()) return err;
            p.gather_of[{fi, c}] = (int)p.gathers.size();
            p.gathers.push_back(std::move(gt));
        }
    if (p.bloch) {
        // no interpolation point may lie across the Bloch-periodic x edge
        // (its weight would need the phase): the unwrapped x index of every
        // point must fall inside the grid
        for (const Face& f : p.faces)
            for (int c = 0; c < kNumComp; ++c)
                for (int smp = 0; smp < f.nsamp; ++smp) {
                    int s2;
                    if (f.axis == 0) {
                        s2 = 2 * f.plane;
                    } else {
                        const int t = f.ntang == 1 ? smp : (f.tang[0] == 0 ? smp / f.count[1] : smp % f.count[1]);
                        const int k = f.tang[0] == 0 ? 0 : 1;
                        s2 = 2 * (f.start[k] + t) + 1;
                    }
                    const int d = s2 - kOffset2[c][0];
                    const int lo = (d % 2 + 2) % 2 == 0 ? d / 2 : (d - 1) / 2;
                    const int hi = (d % 2 + 2) % 2 == 0 ? d / 2 : (d + 1) / 2;
                    if (lo < 0 || hi >= p.nx) return "stress surface reaches across the Bloch-periodic x edge";
                }
    }
    return surface_medium(p);
}

// Medium S lies in: every interpolation point of every gather must hold the
// same eps (E components) and mu (H components), finite and positive.
static std::string surface_medium(Problem& p) {
    std::set<double> e_vals, h_vals;
    for (const Gather& gt : p.gathers) {
        const int c = gt.comp;
        for (int32_t ix : gt.idx) {
            int id = p.ids[c][ix];
            if (is_e(c)) {
                e_vals.insert(id == kWallId ? -INFINITY : p.eps[id]);
                // a dispersive medium would make the stress tensor's eps_S depend on frequency
                if (id != kWallId && p.has_terms(id)) return "stress surface lies in a dispersive material";
            } else {
                h_vals.insert(p.mu[id]);
            }
        }
    }
    if (e_vals.size() != 1 || h_vals.size() != 1)
        return "stress surface does not lie in one uniform medium";
    p.eps_s = *e_vals.begin();
    p.mu_s = *h_vals.begin();
    if (!(std::isfinite(p.eps_s) && p.eps_s > 0 && std::isfinite(p.mu_s) && p.mu_s > 0))
        return "stress surface touches a conductor";
    return "";
}

// Basis and gathers of a cylindrical surface (faces already built).
static std::string finish_cyl_surface(Problem& p, const cf_surface& s) {
    const double dx = 1.0 / p.grid.res;
    p.basis.clear();
    p.labels.clear();
    p.nrows.clear();
    for (const Face& f : p.faces) {
        auto b = weighted_cosine_rows(f.qw, s.n_harm, dx);
        const int rows = (int)(b.size() / f.nsamp);
        std::vector<int> lab(rows);
        for (int r = 0; r < rows; ++r) lab[r] = r;
        p.basis.push_back(std::move(b));
        p.labels.push_back(lab);
        p.nrows.push_back(rows);
    }
    p.gathers.clear();
    p.gather_of.clear();
    for (int fi = 0; fi < (int)p.faces.size(); ++fi)
        for (int c = 0; c < kNumComp; ++c)
            for (int one = 0; one < 2; ++one) {
                Gather gt;
                std::string err = make_gather_cyl(p, fi, c, one == 1, gt);
                if (!err.empty()) return err;
                p.gather_of[{fi, c + (one ? 8 : 0)}] = (int)p.gathers.size();
                p.gathers.push_back(std::move(gt));
            }
    return surface_medium(p);
}

// Stability of the centred Lorentz scheme in a uniform medium (eps_inf, mu,
// terms).  A plane wave with Omega^2 = (4 / dt^2) sin^2(omega dt / 2) and
// curl-curl eigenvalue K^2 / mu obeys
//     Omega^2 (eps_inf + sum d_eps w0^2 / (w0^2 - Omega^2)) = K^2 / mu,
// and is stable when every root Omega^2 <= X = 4 / dt^2.  Above the largest
// w0^2 the left side minus the right increases with Omega^2, so the scheme
// is stable when w0 dt < 2 for every term and
//     eps_inf X - K_max^2 / mu + sum d_eps w0^2 X / (w0^2 - X) > 0,
// K_max^2 = bound / dx^2 (all in units of dx^2 here).
bool lorentz_stable(double eps_inf, double mu, const double* de, const double* w0, int n, double courant,
                    double dx, double bound) {
    const double X = 4.0 / (courant * courant);
    double f = eps_inf * X - bound / mu;
    for (int j = 0; j < n; ++j) {
        if (de[j] == 0.0) continue;
        const double w2 = (w0[j] * dx) * (w0[j] * dx);
        if (w2 * courant * courant >= 4.0) return false;
        f += de[j] * w2 * X / (w2 - X);
    }
    return f > 0.0;
}

std::string validate_opts(const Problem& p, const cf_opts& o, cf_status* code) {
    *code = CF_E_ARG;
    if (!(o.sigma >= 0) || !std::isfinite(o.sigma)) return "sigma must be >= 0";
    if (!(o.courant > 0)) return "courant must be > 0";
    if (o.n_steps < 1) return "n_steps must be >= 1";
    if (o.precision != CF_FP64 && o.precision != CF_FP32) return "unknown precision";
    if (o.path != CF_PATH_BATCHED && o.path != CF_PATH_PLAIN) return "unknown path";
    if (o.kernel != CF_KERNEL_GENERAL && o.kernel != CF_KERNEL_ZINV2D) return "unknown kernel";
    if (p.reduced()) {
        if (o.pol != CF_POL_3D) return "cylindrical and k_z runs take CF_POL_3D (all six components)";
    } else if (p.grid.ndim == 2) {
        if (o.pol < 1 || o.pol > 3) return "2D runs take CF_POL_TM and/or CF_POL_TE";
        if (o.kernel == CF_KERNEL_ZINV2D && !p.vacuum_conductors) {
            *code = CF_E_UNSUPPORTED;
            return "the z-invariant kernel holds for perfect conductors in vacuum only: a material with "
                   "finite eps or mu other than 1 mixes the polarizations at k_z != 0 (use the general "
                   "kernel for the two-dimensional force, or a k_z problem for the force per unit length)";
        }
    } else {
        if (o.pol != CF_POL_3D) return "3D runs take CF_POL_3D";
        if (o.kernel == CF_KERNEL_ZINV2D) {
            *code = CF_E_UNSUPPORTED;
            return "the z-invariant kernel applies to 2D runs only";
        }
    }
    if (p.dispersive && (p.grid.ndim == 3 || p.cyl)) {
        *code = CF_E_UNSUPPORTED;
        return "dispersive materials are implemented for Cartesian 2D and k_z problems";
    }
    if (p.grid.ndim == 3) {
        if (p.grid.bc[0] == CF_BC_PML || p.grid.bc[1] == CF_BC_PML) {
            *code = CF_E_UNSUPPORTED;
            return "3D PML is implemented along z only";
        }
    }
    // Yee stability: dt * v_max * sqrt(ndim) / dx < 1
    double emin = INFINITY;
    for (int i = 0; i < p.nmat; ++i) {
        double e = std::isfinite(p.eps[i]) ? p.eps[i] : INFINITY;
        double m = std::isfinite(p.mu[i]) ? p.mu[i] : INFINITY;
        emin = std::min(emin, e * m);
    }
    if (!std::isfinite(emin)) emin = 1.0;
    double vmax = 1.0 / std::sqrt(emin);
    if (o.courant * vmax * std::sqrt((double)p.grid.ndim) >= 1.0) {
        *code = CF_E_CFL;
        return "courant number above the Yee stability limit";
    }
    if (p.dispersive) {
        // centred Lorentz update: every term needs w0 dt < 2, and the coupled
        // field-polarization frequency of the fastest grid mode must stay
        // below 2 / dt (lorentz_stable)
        double bound = 4.0 * p.grid.ndim;
        if (p.kz) {
            double kmax = 0;
            for (double k : p.kzs) kmax = std::max(kmax, std::abs(k) / p.grid.res);
            bound = 8.0 + kmax * kmax;
        }
        const double dx = 1.0 / p.grid.res;
        for (int i = 0; i < p.nmat; ++i) {
            if (!p.has_terms(i) || !std::isfinite(p.eps[i]) || !std::isfinite(p.mu[i])) continue;
            if (!lorentz_stable(p.eps[i], p.mu[i], &p.lor_de[(size_t)i * p.n_lor], &p.lor_w0[(size_t)i * p.n_lor],
                                p.n_lor, o.courant, dx, bound)) {
                *code = CF_E_CFL;
                return "a Lorentz medium is unstable at this time step (the coupled field and polarization "
                       "frequency exceeds 2 / dt): lower the Courant number";
            }
        }
    }
    if (p.cyl && o.courant * vmax > 0.5) {
        *code = CF_E_CFL;
        return "cylindrical runs need courant * max speed <= 0.5";
    }
    if (p.kz) {
        double kmax = 0;
        for (double k : p.kzs) kmax = std::max(kmax, std::abs(k) / p.grid.res);
        if (o.courant * vmax * std::sqrt(8.0 + kmax * kmax) / 2.0 >= 1.0) {
            *code = CF_E_CFL;
            return "courant number above the stability limit of the largest k_z";
        }
    }
    *code = CF_OK;
    return "";
}

// Stress-tensor channels for force axis d and a face with normal a
// (Minkowski tensor with the medium's eps_S, mu_S):
//   a == d: E(k->k) eps_S (delta_kd - 1/2), H(k->k) mu_S (delta_kd - 1/2)
//   a != d: E(a->d) eps_S and H(a->d) mu_S when both components exist.
std::vector<Channel> channel_table(const Problem& p, int pol_mask) {
    std::vector<Channel> out;
    const int d = p.surf.force_axis;
    std::vector<int> pols;
    if (p.grid.ndim == 3 || p.reduced()) {
        pols = {CF_POL_3D};
    } else {
        if (pol_mask & CF_POL_TM) pols.push_back(CF_POL_TM);
        if (pol_mask & CF_POL_TE) pols.push_back(CF_POL_TE);
    }
    for (int pol : pols) {
        std::vector<int> e, h;
        pol_components(pol, e, h);
        auto has = [](const std::vector<int>& v, int c) {
            return std::find(v.begin(), v.end(), c) != v.end();
        };
        for (int fi = 0; fi < (int)p.faces.size(); ++fi) {
            const Face& f = p.faces[fi];
            const int a = f.axis;
            struct Spec { int kind, src, meas; double coef; };
            std::vector<Spec> specs;
            if (a == d) {
                for (int c : e) specs.push_back({0, c, c, p.eps_s * ((c == d ? 1.0 : 0.0) - 0.5)});
                for (int c : h) specs.push_back({1, c, c, p.mu_s * ((c - 3 == d ? 1.0 : 0.0) - 0.5)});
            } else {
                if (has(e, a) && has(e, d)) specs.push_back({0, a, d, p.eps_s});
                if (has(h, 3 + a) && has(h, 3 + d)) specs.push_back({1, 3 + a, 3 + d, p.mu_s});
            }
            for (int r = 0; r < p.nrows[fi]; ++r)
                for (const Spec& sp : specs) {
                    Channel ch;
                    ch.face = fi;
                    ch.row = r;
                    ch.label = p.labels[fi][r];
                    ch.kind = sp.kind;
                    ch.pol = pol;
                    ch.src = sp.src;
                    ch.meas = sp.meas;
                    ch.sign = (double)f.side * sp.coef;
                    out.push_back(ch);
                }
        }
    }
    if (p.reduced()) {
        // order-major: the channel set once per order (azimuthal order m,
        // weight 1 for m = 0 and 2 above: the -m term is the conjugate of
        // the +m term; or k_z point q with its quadrature weight) with the
        // weight in the sign
        const std::vector<Channel> base = std::move(out);
        out.clear();
        for (int q = 0; q < p.n_orders(); ++q)
            for (Channel ch : base) {
                ch.order = q;
                ch.label += q * p.surf.n_harm;
                ch.sign *= p.order_weight(q);
                out.push_back(ch);
            }
    }
    return out;
}

// Time-centred conductivity: a lossy component of a channel's kind gets
// a = (1 - r)/(1 + r), b = S_c/(eps or mu)/(1 + r), r = sigma dt / 2; the
// other field of the run is lossless (a = 1, b = S_c/(eps or mu)).  A
// conductor (PEC for E, PMC for H, or a wall E component) gets a = b = 0.
std::vector<double> coefficient_lut(const Problem& p, double sigma, double courant) {
    std::vector<double> lut(2 * kNumComp * 256 * 2, 0.0);
    const double dt = courant / p.grid.res;
    const double r = 0.5 * sigma * dt;
    const double la = (1.0 - r) / (1.0 + r), lb = 1.0 / (1.0 + r);
    for (int kind = 0; kind < 2; ++kind)
        for (int c = 0; c < kNumComp; ++c)
            for (int id = 0; id < 256; ++id) {
                double a = 0, b = 0;
                bool valid = id < p.nmat || (id == kWallId && is_e(c));
                if (valid) {
                    double v;
                    if (is_e(c)) v = id == kWallId ? -INFINITY : p.eps[id];
                    else v = p.mu[id];
                    if (std::isfinite(v)) {
                        bool lossy = (kind == 0) == is_e(c);
                        a = lossy ? la : 1.0;
                        b = lossy ? courant / v * lb : courant / v;
                    }
                }
                size_t at = ((size_t)(kind * kNumComp + c) * 256 + id) * 2;
                lut[at] = a;
                lut[at + 1] = b;
            }
    return lut;
}

// K(t) = 2 pi Im g(-t).  General form: the Laplace integral
// int_0^inf (k + s/2) sqrt(1 + s/k) e^{-k t} dk, which the substitution
// k + s/2 = (s/2) cosh u turns into (s^2/4) int_0^inf cosh u (cosh u + 1)
// e^{-x (cosh u - 1)} du with x = s t / 2; the integrand is entire and
// decays double-exponentially, so the trapezoidal rule in u converges
// geometrically.  Near u = 0 the integrand behaves like exp(-x u^2 / 2), so
// the step is min(1/8, 1/(2 sqrt(x))): both bounds keep the aliasing error
// below exp(-70).
// z-invariant 2D form: 1/t^3 + 3 s/(4 t^2) + s^2/(4 t).
static double k_general(double t, double s) {
    if (s == 0.0) return 1.0 / (t * t);
    const double x = 0.5 * s * t;
    const double h = std::min(0.125, 0.5 / std::sqrt(x));
    double sum = 0.5 * 2.0;   // u = 0: cosh 0 (cosh 0 + 1) = 2, half weight
    for (int k = 1;; ++k) {
        double u = k * h;
        double c = std::cosh(u);
        double arg = x * (c - 1.0);
        double term = c * (c + 1.0) * std::exp(-arg);
        sum += term;
        if (arg > 50.0 && term < 1e-18 * sum) break;
        if (k > 100000) break;
    }
    return 0.25 * s * s * h * sum;
}

// CPML profile (Roden-Gedney with kappa = 1, alpha = 0): in the layers of
// P cells at both ends of z, sigma_p(z) = sigma_max (depth / P)^3 with
// depth the distance in cells from the layer's inner face and
// sigma_max = -(3 + 1) ln(1e-8) / (2 P dx); b = exp(-sigma_p dt), c = b - 1.
void pml_tables(const Problem& p, double courant, std::vector<double>& bh, std::vector<double>& ch,
                std::vector<double>& be, std::vector<double>& ce) {
    const int nz = p.nz, P = p.grid.bc[2] == CF_BC_PML ? p.grid.pml_cells[2] : 0;
    bh.assign(nz, 1.0);
    ch.assign(nz, 0.0);
    be.assign(nz, 1.0);
    ce.assign(nz, 0.0);
    if (P <= 0) return;
    const double dx = 1.0 / p.grid.res, dt = courant * dx;
    const double smax = -(3.0 + 1.0) * std::log(1e-8) / (2.0 * P * dx);
    for (int k = 0; k < nz; ++k)
        for (int half = 0; half < 2; ++half) {
            const double z = k + 0.5 * half;
            const double depth = std::max(std::max(P - z, z - (nz - P)), 0.0);
            const double sg = smax * std::pow(depth / P, 3);
            const double b = std::exp(-sg * dt);
            if (half) {
                bh[k] = b;
                ch[k] = b - 1.0;
            } else {
                be[k] = b;
                ce[k] = b - 1.0;
            }
        }
}

// The same profile along in-plane axis `axis` of a 2D problem: appends
// b, c at the half-cell positions, then b, c at the integer positions (n
// values each); nothing when the axis has no layers.
void pml_axis_tables(const Problem& p, int axis, double courant, std::vector<double>& out) {
    if (p.grid.bc[axis] != CF_BC_PML) return;
    const int n = axis == 0 ? p.nx : p.ny, P = p.grid.pml_cells[axis];
    const double dx = 1.0 / p.grid.res, dt = courant * dx;
    const double smax = -(3.0 + 1.0) * std::log(1e-8) / (2.0 * P * dx);
    const size_t o = out.size();
    out.resize(o + 4 * (size_t)n);
    for (int half = 1; half >= 0; --half)
        for (int q = 0; q < n; ++q) {
            const double x = q + 0.5 * half;
            const double depth = std::max(std::max(P - x, x - (n - P)), 0.0);
            const double b = std::exp(-smax * std::pow(depth / P, 3) * dt);
            const size_t row = o + (half ? 0 : 2 * (size_t)n);
            out[row + q] = b;
            out[row + n + q] = b - 1.0;
        }
}

void kernel_table(int kernel, double sigma, double dt, int n, double* out) {
    for (int m = 1; m <= n; ++m) {
        double t = m * dt;
        if (kernel == CF_KERNEL_ZINV2D)
            out[m - 1] = 1.0 / (t * t * t) + 0.75 * sigma / (t * t) + 0.25 * sigma * sigma / t;
        else
            out[m - 1] = k_general(t, sigma);
    }
}

}  // namespace cf
