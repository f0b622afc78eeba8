// Host-side problem description and solve planning.
//
// A cf_problem holds the copied inputs plus everything derived from them that
// does not depend on the run options: wall-marked material ids, the faces of
// the stress surface S, the interpolation (gather) tables of every
// (face, component) pair, the per-face cosine basis and the medium S lies in.
// A SolvePlan adds what depends on the options: the channel table, the
// coefficient look-up tables and the time kernel samples.
#pragma once

#include <cstdint>
#include <map>
#include <string>
#include <utility>
#include <vector>

#include "../../include/casimir_fdtd.h"

namespace cf {

constexpr int kWallId = 255;        // E components on a PEC(-backed) wall
constexpr int kNumComp = 6;          // Ex Ey Ez Hx Hy Hz

// doubled Yee offsets (x, y, z) of each component
extern const int kOffset2[kNumComp][3];

struct Face {
    int index;        // 2*axis + (side > 0)
    int axis;         // normal axis
    int side;         // -1 / +1
    int plane;        // integer coordinate of the plane
    int ntang;        // tangential axes (1 in 2D, 2 in 3D)
    int tang[2];
    int start[2];
    int count[2];
    int nsamp;
    // cylindrical faces: doubled coordinate of the plane along the normal
    // axis, doubled tangential coordinate and quadrature weight per sample
    int plane2 = 0;
    std::vector<int> samp2;
    std::vector<double> qw;
};

// Interpolation W of one component on one face: for sample s, points
// idx[s*P + p] with weights w[s*P + p].  The adjoint (scatter) form lists the
// distinct grid points with the (sample, weight) pairs that touch them.
struct Gather {
    int face, comp, P, nsamp;
    std::vector<int32_t> idx;
    std::vector<double> w;
    std::vector<int32_t> uidx;    // distinct grid points
    std::vector<int32_t> uoff;    // CSR offsets into usamp/uw (size uidx+1)
    std::vector<int32_t> usamp;
    std::vector<double> uw;
};

struct Channel {
    int face, row, label;
    int kind;        // 0: E-current source, 1: H-current source
    int pol;         // CF_POL_TM / CF_POL_TE / CF_POL_3D
    int src, meas;   // component ids
    double sign;
    int order = 0;   // azimuthal order m (cylindrical problems)
};

struct Problem {
    uint64_t uid = 0;                         // unique per created problem (copies share it)
    cf_grid grid{};
    int nx = 0, ny = 0, nz = 0;
    int64_t ncell = 0;
    int nmat = 0;
    std::vector<double> eps, mu;
    std::vector<uint8_t> ids[kNumComp];
    cf_surface surf{};
    std::vector<Face> faces;
    std::vector<std::vector<double>> basis;   // per face: rows x nsamp
    std::vector<std::vector<int>> labels;     // per face: label per row
    std::vector<int> nrows;
    std::map<std::pair<int, int>, int> gather_of;   // (face, gather_key) -> gathers index
    std::vector<Gather> gathers;
    double eps_s = 0, mu_s = 0;
    bool cyl = false;                         // cylindrical (r, z) problem
    bool kz = false;                          // z-invariant problem at Bloch wavevectors k_z
    int m_max = 0;
    std::vector<double> kzs, kz_w;            // k_z points and weights
    std::vector<double> kxs;                  // Bloch wavevector along x per point (k_z problems)
    bool bloch = false;                       // complex fields: some kx != 0
    // every material the grid uses is vacuum (eps = mu = 1) or a perfect
    // electric / magnetic conductor (the premise of the z-invariant kernel)
    bool vacuum_conductors = true;
    // Lorentz terms (d_eps, w0) of each material, n_lor per material
    // (nmat x n_lor, row-major); dispersive: some material the grid uses has
    // a term with d_eps != 0 (not a conductor)
    int n_lor = 0;
    std::vector<double> lor_de, lor_w0;
    bool dispersive = false;
    bool has_terms(int id) const {
        if (id >= nmat) return false;
        for (int j = 0; j < n_lor; ++j)
            if (lor_de[(size_t)id * n_lor + j] != 0.0) return true;
        return false;
    }
    // reduced two-dimensional problems: six components, one run per order
    // (azimuthal order m, or k_z point q)
    bool reduced() const { return cyl || kz; }
    // a 2D problem with CPML layers on an in-plane axis (split kernels only)
    bool pml2d() const { return grid.ndim == 2 && (grid.bc[0] == CF_BC_PML || grid.bc[1] == CF_BC_PML); }
    // a Cartesian 2D problem the fused kernel can take (no polarizations, no CPML)
    bool fusable2d() const { return grid.ndim == 2 && !reduced() && !dispersive && !pml2d(); }
    int n_orders() const { return cyl ? m_max + 1 : kz ? (int)kzs.size() : 1; }
    double order_weight(int q) const { return cyl ? (q == 0 ? 1.0 : 2.0) : kz ? kz_w[q] : 1.0; }
    // coupling of order q in the undivided curls: m, or k dx
    double coupling(int q) const { return cyl ? (double)q : kz ? kzs[q] / grid.res : 0.0; }
};

// Key of a (face, component) gather: cylindrical problems keep a second
// table per component for order m = 1, whose axis values of E_r and H_phi
// are the next row's (every other order reads zero there).
inline int gather_key(const Problem& p, int comp, int order) {
    return comp + (p.cyl && order == 1 ? 8 : 0);
}

// Courant number and step count of azimuthal order m (cylindrical
// problems); Cartesian problems run every channel on (courant, n_steps).
double order_courant(const Problem& p, double courant, int m);
int order_steps(const Problem& p, const cf_opts& o, int m);
int max_steps(const Problem& p, const cf_opts& o);
int n_comp(const Problem& p);
int harmonic_len(const Problem& p);

// Components of each polarization: (E list, H list) as component ids.
void pol_components(int pol, std::vector<int>& e, std::vector<int>& h);
// Slot position of component `comp` inside a channel's field block.
int comp_slot(int pol, int comp);
int n_comp_for(int ndim);

std::string build_problem(const cf_grid& g, const cf_materials& m, const cf_surface& s,
                          Problem& p);   // returns "" or an error message
std::string validate_opts(const Problem& p, const cf_opts& o, cf_status* code);
std::vector<Channel> channel_table(const Problem& p, int pol_mask);

// coefficient tables: lut[(kind*6 + comp)*256 + id] = (a, b)
std::vector<double> coefficient_lut(const Problem& p, double sigma, double courant);

// K(t_m), m = 1..n
void kernel_table(int kernel, double sigma, double dt, int n, double* out);

// CPML along z: b, c at the z positions of H_x/H_y (k + 1/2) and E_x/E_y (k).
void pml_axis_tables(const Problem& p, int axis, double courant, std::vector<double>& out);
void pml_tables(const Problem& p, double courant, std::vector<double>& bh, std::vector<double>& ch,
                std::vector<double>& be, std::vector<double>& ce);

}  // namespace cf
