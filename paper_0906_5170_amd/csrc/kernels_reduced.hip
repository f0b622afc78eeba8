// Reduced two-dimensional Yee updates: six components on a 2D grid, one
// run per "order", for
//   - cylindrically symmetric problems (Sec. III C; Appendix, harmonic
//     expansion in cylindrical coordinates), one run per azimuthal order m;
//   - z-invariant problems at a Bloch wavevector k along z (Sec. III B, one
//     2D simulation per k_z), optionally Bloch-periodic along x (Sec. III D,
//     complex fields).
//
// Cylindrical.  Fields proportional to exp(i m phi), with E_phi, H_r, H_z
// carried as -i times their value, obey the real system
//   mu  dh_r/dt   = -[ (m/r) e_z - d_z e_phi ]
//   mu  dh_phi/dt = -[ d_z e_r - d_r e_z ]
//   mu  dh_z/dt   = -[ (1/r) d_r (r e_phi) - (m/r) e_r ]
//   eps de_r/dt   =    -(m/r) h_z - d_z h_phi
//   eps de_phi/dt =    d_z h_r - d_r h_z
//   eps de_z/dt   =    (1/r) d_r (r h_phi) + (m/r) h_r
// The axial coordinate is the grid's x (index i), the radius its y (index j):
// slots Ex = e_z, Ey = e_r, Ez = e_phi, Hx = h_z, Hy = h_r, Hz = h_phi, each
// an (nr x nz) array, z fastest.  Ey, Hx, Hz sit at r = j cells, Ex, Ez, Hy
// at r = j - 1/2 (their row 0 lies outside and stays 0).  The tube wall is
// at r = nr - 1/2: a neighbour beyond it reads 0.  Along z a neighbour beyond
// the grid reads 0 (PEC ends) or wraps (periodic).  Axis (row 0 of Ey, Hx,
// Hz): h_z there follows the circulation of e_phi around the disk of radius
// 1/2 cell, (4 / dx) e_phi(r = 1/2), for m = 0 and is 0 otherwise; e_r and
// h_phi enter no update there and are kept at 0 (the surface interpolation
// applies their axis value, the next row's for m = 1).
//
// k_z.  With E_z, H_x, H_y carried as -i times their value the same forms
// hold with m/r -> k and unit radial weights (Cartesian x, y; both walls
// PEC or periodic).  Bloch-periodic x (CPLX): real and imaginary parts in
// two six-component blocks, mixed only by the phase of the neighbour read
// across the periodic x edge.
//
// Coefficients (a, b) come from the Cartesian per-kind tables built for
// the order's Courant number: x <- a x -/+ b curl, with the curls above in
// undivided form (times dx).
//
// Drivers, all evaluating the same per-cell value functions (their fields
// agree bitwise): split half-step launches (one launch per half step for the
// channels of one order), and the resident solve, where one block carries
// one channel through clear, kick, start and all its steps with the surface
// projection, in a single launch for channels of any mix of orders, with the
// fields in registers (LDS neighbour exchange) or in global memory (a
// channel's block stays in the L2 of its XCD).
#include <mutex>
#include <type_traits>

#include "../../include/casimir_fdtd.h"
#include "device.hpp"
#include "red_span.hpp"
#include "yee_common.hpp"

namespace cf {

namespace {

constexpr int BX = 64;
constexpr int BY = 4;
constexpr int kResThreads = 1024;

using yee::lut_ab;

inline dim3 grid_red(const Grid2D& g, int nslots) {
    const int tiles = ((g.nx + BX - 1) / BX) * ((g.ny + BY - 1) / BY);
    return dim3(tiles, nslots, 1);
}

// Reduced update, with M the coupling of the run (m, or k dx) and the curls
// in undivided form:
//   h_x/h_z: ((A e_z(j+1) - B e_z) - M e_y) C       h_y/h_r: M e_x D - d_x e_z
//   e_x/e_z: ((P h_z - Q h_z(j-1)) + M h_y) D       e_y/e_r: -M h_x C - d_x h_z
//   h_z/h_phi and e_z/e_phi: the Cartesian two-dimensional forms;
// cylindrical (CYL): (A, B, C, D, P, Q) = (j + 1/2, j - 1/2, 1/j, 1/(j - 1/2),
// j, j - 1), row 0 the axis with its own rules; k_z: all 1.  The row table
// holds 6 values per row (field precision); the kernels read C and D from it
// and form the others from j.
enum { RA = 0, RB, RC, RD, RP, RQ, kRowFactors };

// Updated h components (hx, hy, hz) of a cell at row j from its own fields,
// the neighbours e(j+1) (ezu, exu) and e(i+1) (ezr, eyr) and the (a, b)
// pairs lx, ly, lz: MODE 0 h <- a h - b curl e, MODE 1 the consistent start
// h^{-1/2} = (b / 2) curl e^0.  axis: row 0 is the symmetry axis
// (cylindrical).  Every driver evaluates these forms, so their fields agree
// bitwise.
template <typename T, int MODE, bool CYL>
__device__ __forceinline__ void h_values(T& hx, T& hy, T& hz, T ex, T ey, T ez, T ezu, T exu, T ezr, T eyr,
                                         const T* lx, const T* ly, const T* lz, T M, int j, const T* rw) {
    T cz, cr;
    if (CYL) {
        if (j == 0) {
            // axis: h_z from the disk circulation (m = 0), h_r outside, h_phi 0
            const T c4 = T(4) * ezu;
            if (MODE == 0) hx = M == T(0) ? yee::sub(lx[0], hx, lx[1], c4) : T(0);
            else hx = M == T(0) ? yee::half(lx[1], c4) : T(0);
            hy = T(0);
            hz = T(0);
            return;
        }
        const T r = T(j);
        cz = (((r + T(0.5)) * ezu - (r - T(0.5)) * ez) - M * ey) * rw[RC];
        cr = (M * ex) * rw[RD] - (ezr - ez);
    } else {
        cz = (ezu - ez) - M * ey;
        cr = M * ex - (ezr - ez);
    }
    const T cp = (eyr - ey) - (exu - ex);
    if (MODE == 0) {
        hx = yee::sub(lx[0], hx, lx[1], cz);
        hy = yee::sub(ly[0], hy, ly[1], cr);
        hz = yee::sub(lz[0], hz, lz[1], cp);
    } else {
        hx = yee::half(lx[1], cz);
        hy = yee::half(ly[1], cr);
        hz = yee::half(lz[1], cp);
    }
}

// Updated e components (ex, ey, ez) of a cell at row j from its own fields
// and the neighbours h(j-1) (hxd, hzd) and h(i-1) (hyl, hzl): MODE 0
// e <- a e + b curl h, MODE 1 the consistent start e^{+1/2} = (b / 2) curl h^0.
template <typename T, int MODE, bool CYL>
__device__ __forceinline__ void e_values(T& ex, T& ey, T& ez, T hx, T hy, T hz, T hxd, T hzd, T hyl, T hzl,
                                         const T* lx, const T* ly, const T* lz, T M, int j, const T* rw) {
    T cz, cr;
    if (CYL) {
        if (j == 0) {
            // e_z, e_phi outside / on the wall id, e_r on the axis: all 0
            ex = T(0);
            ey = T(0);
            ez = T(0);
            return;
        }
        const T r = T(j);
        cz = ((r * hz - (r - T(1)) * hzd) + M * hy) * rw[RD];
        cr = -((M * hx) * rw[RC]) - (hz - hzl);
    } else {
        cz = (hz - hzd) + M * hy;
        cr = -(M * hx) - (hz - hzl);
    }
    const T cp = (hy - hyl) - (hx - hxd);
    if (MODE == 0) {
        ex = yee::add(lx[0], ex, lx[1], cz);
        ey = yee::add(ly[0], ey, ly[1], cr);
        ez = yee::add(lz[0], ez, lz[1], cp);
    } else {
        ex = yee::half(lx[1], cz);
        ey = yee::half(ly[1], cr);
        ez = yee::half(lz[1], cp);
    }
}

// The CPML-stretched difference of yee::pml_d2 in two phases, for a cell
// that stretches several differences: pml_fetch issues the loads of one
// difference's (b, c) and psi (none outside the layers), pml_apply forms
// psi <- b psi + c D, stores it and returns D + psi, the same arithmetic.
// Fetching every difference of a cell before applying any keeps all their
// loads in flight together; a psi store between them would hold the next
// difference's loads back (the compiler cannot tell that the psi entries
// are distinct, which they are: each difference has its own slot and axis).
template <typename T>
struct PmlTerm {
    T* at;   // nullptr: outside the layers
    double b, c;
    T psi;
};
// The loads are unconditional for every lane, with or without layers on the
// axis (a lane outside the layers reads the first table entry and the first
// psi entry of the channel's block and discards them), so that no load sits
// under a branch: the compiler would wait for it before the branches merge.
// psi must be the channel's CPML block (not null).  Every read stays inside
// the CPML profile region, which holds 4 (nx + ny) values per order for both
// axes whatever their layers (the host's layout).
template <typename T>
__device__ __forceinline__ PmlTerm<T> pml_fetch(const Grid2D& g, T* psi, int slot, int axis, bool half, int i,
                                                int j) {
    PmlTerm<T> t;
    const int P = g.pml[axis];
    const int n = axis == 0 ? g.nx : g.ny;
    const int q = axis == 0 ? i : j;
    const bool in = P > 0 && (q < P || q >= n - P);
    const int qc = in ? q : 0;
    const int qq = in ? (q < P ? q : q - (n - 2 * P)) : 0;
    T* arr = psi + slot * g.psi_slot + (axis == 0 ? 0 : (int64_t)g.ny * 2 * g.pml[0]);
    const double* tab = g.pml_tab[axis] + (half ? 0 : 2 * n);
    T* at = in ? arr + (axis == 0 ? (int64_t)j * (2 * P) + qq : (int64_t)qq * g.nx + i) : psi;
    t.b = tab[qc];
    t.c = tab[n + qc];
    t.psi = *at;
    t.at = in ? at : nullptr;
    return t;
}
template <typename T>
__device__ __forceinline__ T pml_apply(const PmlTerm<T>& t, T D) {
    if (t.at == nullptr) return D;
    const T p = fma(T(t.b), t.psi, T(t.c) * D);
    *t.at = p;
    return D + p;
}

// The k_z forms (no cylindrical weights) with the in-plane differences
// passed in, as the CPML stretches them (split kernels only): the same
// operations as h_values / e_values with CYL = false (MODE 0 the step,
// MODE 1 the consistent start).
template <typename T, int MODE>
__device__ __forceinline__ void h_values_kz(T& hx, T& hy, T& hz, T ex, T ey, T dy_ez, T dx_ez, T dx_ey, T dy_ex,
                                            const T* lx, const T* ly, const T* lz, T M) {
    const T cz = dy_ez - M * ey, cr = M * ex - dx_ez, cp = dx_ey - dy_ex;
    if (MODE == 0) {
        hx = yee::sub(lx[0], hx, lx[1], cz);
        hy = yee::sub(ly[0], hy, ly[1], cr);
        hz = yee::sub(lz[0], hz, lz[1], cp);
    } else {
        hx = yee::half(lx[1], cz);
        hy = yee::half(ly[1], cr);
        hz = yee::half(lz[1], cp);
    }
}
template <typename T, int MODE>
__device__ __forceinline__ void e_values_kz(T& ex, T& ey, T& ez, T hx, T hy, T dy_hz, T dx_hz, T dx_hy, T dy_hx,
                                            const T* lx, const T* ly, const T* lz, T M) {
    const T cz = dy_hz + M * hy, cr = -(M * hx) - dx_hz, cp = dx_hy - dy_hx;
    if (MODE == 0) {
        ex = yee::add(lx[0], ex, lx[1], cz);
        ey = yee::add(ly[0], ey, ly[1], cr);
        ez = yee::add(lz[0], ez, lz[1], cp);
    } else {
        ex = yee::half(lx[1], cz);
        ey = yee::half(ly[1], cr);
        ez = yee::half(lz[1], cp);
    }
}

// Reduced-update parameters of one run: coupling M, the row factors and,
// for complex (Bloch-periodic x) runs, the phase p = pc + i ps that a field
// gains across the periodic x edge.
template <typename T>
struct RedRun {
    T M;
    const T* rows;
    T pc, ps;
};

// Complex runs keep the real part of the six components in the first
// 6 x ncell values of a channel block and the imaginary part in the next.
// The x neighbour across the periodic edge of part `part` (0 real, 1
// imaginary): forward (F[nx] = p F[0]) or backward (F[-1] = conj(p) F[nx-1]),
// from the wrapped cell's own-part value a and other-part value b.
template <typename T>
__device__ __forceinline__ T bloch_fwd(T a, T b, int part, T pc, T ps) {
    return part == 0 ? a * pc - b * ps : a * pc + b * ps;
}
template <typename T>
__device__ __forceinline__ T bloch_bwd(T a, T b, int part, T pc, T ps) {
    return part == 0 ? a * pc + b * ps : a * pc - b * ps;
}

// H update of cell (i, j), part `part`, of the channel block F in global memory.
// psi: the channel's CPML block (k_z runs with in-plane layers), or nullptr.
template <typename T, int MODE, bool CYL, bool CPLX = false>
__device__ __forceinline__ void hred_cell(T* __restrict__ F, const Grid2D& g, const T* __restrict__ lut, int kind,
                                          const RedRun<T>& rr, int i, int j, int part = 0, T* psi = nullptr) {
    T* const Fo = F + (CPLX ? (1 - part) * 6 * g.ncell : 0);    // the other part (complex runs)
    F += CPLX ? part * 6 * g.ncell : 0;
    const T* Ex = F;
    const T* Ey = F + g.ncell;
    const T* Ez = F + 2 * g.ncell;
    T* Hx = F + 3 * g.ncell;
    T* Hy = F + 4 * g.ncell;
    T* Hz = F + 5 * g.ncell;
    const int64_t c = (int64_t)j * g.nx + i;
    const bool in_r = i + 1 < g.nx, in_u = j + 1 < g.ny;
    const int64_t cu = in_u ? c + g.nx : i;                     // row above (wrapped when periodic)
    const bool has_u = in_u || (!CYL && g.pery);   // the tube wall is never periodic
    const T ezu = has_u ? Ez[cu] : T(0);
    const T exu = has_u ? Ex[cu] : T(0);
    T ezr, eyr;
    if (in_r) {
        ezr = Ez[c + 1];
        eyr = Ey[c + 1];
    } else if (!g.perx) {
        ezr = eyr = T(0);
    } else if (CPLX) {
        const int64_t w = c + 1 - g.nx;
        ezr = bloch_fwd(Ez[w], Fo[2 * g.ncell + w], part, rr.pc, rr.ps);
        eyr = bloch_fwd(Ey[w], Fo[g.ncell + w], part, rr.pc, rr.ps);
    } else {
        ezr = Ez[c + 1 - g.nx];
        eyr = Ey[c + 1 - g.nx];
    }
    T hx = Hx[c], hy = Hy[c], hz = Hz[c];
    if (!CYL && psi != nullptr) {
        // CPML: slots Hx 3, Hy 4, Hz 5; H components at half-cell positions
        T* pp = psi + (CPLX ? part * 6 * g.psi_slot : 0);
        const T ex = Ex[c], ey = Ey[c], ez = Ez[c];
        const PmlTerm<T> t0 = pml_fetch(g, pp, 3, 1, true, i, j), t1 = pml_fetch(g, pp, 4, 0, true, i, j);
        const PmlTerm<T> t2 = pml_fetch(g, pp, 5, 0, true, i, j), t3 = pml_fetch(g, pp, 5, 1, true, i, j);
        const T* lx = lut_ab(lut, kind, CF_HX, g.ids[CF_HX][c]);
        const T* ly = lut_ab(lut, kind, CF_HY, g.ids[CF_HY][c]);
        const T* lz = lut_ab(lut, kind, CF_HZ, g.ids[CF_HZ][c]);
        const T d0 = pml_apply(t0, ezu - ez), d1 = pml_apply(t1, ezr - ez);
        const T d2 = pml_apply(t2, eyr - ey), d3 = pml_apply(t3, exu - ex);
        h_values_kz<T, MODE>(hx, hy, hz, ex, ey, d0, d1, d2, d3, lx, ly, lz, rr.M);
    } else if (CYL && psi != nullptr && j > 0) {
        // CPML at the tube ends (along the axis, the grid's x): the axial
        // differences of h_r (slot 4) and h_phi (slot 5) are stretched; the
        // rest is h_values' cylindrical form (the axis row takes h_values)
        const T ex = Ex[c], ey = Ey[c], ez = Ez[c];
        const T* rw = rr.rows + kRowFactors * j;
        const T r = T(j);
        const T cz = (((r + T(0.5)) * ezu - (r - T(0.5)) * ez) - rr.M * ey) * rw[RC];
        const PmlTerm<T> t1 = pml_fetch(g, psi, 4, 0, true, i, j), t2 = pml_fetch(g, psi, 5, 0, true, i, j);
        const T* lx = lut_ab(lut, kind, CF_HX, g.ids[CF_HX][c]);
        const T* ly = lut_ab(lut, kind, CF_HY, g.ids[CF_HY][c]);
        const T* lz = lut_ab(lut, kind, CF_HZ, g.ids[CF_HZ][c]);
        const T cr = (rr.M * ex) * rw[RD] - pml_apply(t1, ezr - ez);
        const T cp = pml_apply(t2, eyr - ey) - (exu - ex);
        if (MODE == 0) {
            hx = yee::sub(lx[0], hx, lx[1], cz);
            hy = yee::sub(ly[0], hy, ly[1], cr);
            hz = yee::sub(lz[0], hz, lz[1], cp);
        } else {
            hx = yee::half(lx[1], cz);
            hy = yee::half(ly[1], cr);
            hz = yee::half(lz[1], cp);
        }
    } else {
        h_values<T, MODE, CYL>(hx, hy, hz, Ex[c], Ey[c], Ez[c], ezu, exu, ezr, eyr,
                          lut_ab(lut, kind, CF_HX, g.ids[CF_HX][c]), lut_ab(lut, kind, CF_HY, g.ids[CF_HY][c]),
                          lut_ab(lut, kind, CF_HZ, g.ids[CF_HZ][c]), rr.M, j, rr.rows + kRowFactors * j);
    }
    Hx[c] = hx;
    Hy[c] = hy;
    Hz[c] = hz;
}

// E update of cell (i, j), part `part`, of the channel block F in global memory.
// psi: as in hred_cell; aux: the channel's polarization block (dispersive
// k_z runs), or nullptr.
template <typename T, int MODE, bool CYL, bool CPLX = false>
__device__ __forceinline__ void ered_cell(T* __restrict__ F, const Grid2D& g, const T* __restrict__ lut, int kind,
                                          const RedRun<T>& rr, int i, int j, int part = 0, T* psi = nullptr,
                                          T* aux = nullptr) {
    T* const Fo = F + (CPLX ? (1 - part) * 6 * g.ncell : 0);
    F += CPLX ? part * 6 * g.ncell : 0;
    T* Ex = F;
    T* Ey = F + g.ncell;
    T* Ez = F + 2 * g.ncell;
    const T* Hx = F + 3 * g.ncell;
    const T* Hy = F + 4 * g.ncell;
    const T* Hz = F + 5 * g.ncell;
    const int64_t c = (int64_t)j * g.nx + i;
    const bool in_d = j > 0;
    const int64_t cd = in_d ? c - g.nx : c + g.ncell - g.nx;    // row below (wrapped when periodic)
    const bool has_d = in_d || (!CYL && g.pery);
    const T hxd = has_d ? Hx[cd] : T(0);
    const T hzd = has_d ? Hz[cd] : T(0);
    T hyl, hzl;
    if (i > 0) {
        hyl = Hy[c - 1];
        hzl = Hz[c - 1];
    } else if (!g.perx) {
        hyl = hzl = T(0);
    } else if (CPLX) {
        const int64_t w = c - 1 + g.nx;
        hyl = bloch_bwd(Hy[w], Fo[4 * g.ncell + w], part, rr.pc, rr.ps);
        hzl = bloch_bwd(Hz[w], Fo[5 * g.ncell + w], part, rr.pc, rr.ps);
    } else {
        hyl = Hy[c - 1 + g.nx];
        hzl = Hz[c - 1 + g.nx];
    }
    T ex = Ex[c], ey = Ey[c], ez = Ez[c];
    // the material ids are read once: a byte load after a field store would
    // have to be repeated (bytes may alias anything)
    const int id_x = g.ids[CF_EX][c], id_y = g.ids[CF_EY][c], id_z = g.ids[CF_EZ][c];
    const T* lx = lut_ab(lut, kind, CF_EX, id_x);
    const T* ly = lut_ab(lut, kind, CF_EY, id_y);
    const T* lz = lut_ab(lut, kind, CF_EZ, id_z);
    if (!CYL && psi != nullptr) {
        // CPML: slots Ex 0, Ey 1, Ez 2; E components at integer positions
        T* pp = psi + (CPLX ? part * 6 * g.psi_slot : 0);
        const T hx = Hx[c], hy = Hy[c], hz = Hz[c];
        const PmlTerm<T> t0 = pml_fetch(g, pp, 0, 1, false, i, j), t1 = pml_fetch(g, pp, 1, 0, false, i, j);
        const PmlTerm<T> t2 = pml_fetch(g, pp, 2, 0, false, i, j), t3 = pml_fetch(g, pp, 2, 1, false, i, j);
        const T d0 = pml_apply(t0, hz - hzd), d1 = pml_apply(t1, hz - hzl);
        const T d2 = pml_apply(t2, hy - hyl), d3 = pml_apply(t3, hx - hxd);
        e_values_kz<T, MODE>(ex, ey, ez, hx, hy, d0, d1, d2, d3, lx, ly, lz, rr.M);
    } else if (CYL && psi != nullptr && j > 0) {
        // CPML at the tube ends: the axial differences of e_r (slot 1) and
        // e_phi (slot 2) are stretched; the rest is e_values' cylindrical form
        const T hx = Hx[c], hy = Hy[c], hz = Hz[c];
        const T* rw = rr.rows + kRowFactors * j;
        const T r = T(j);
        const T cz = ((r * hz - (r - T(1)) * hzd) + rr.M * hy) * rw[RD];
        const PmlTerm<T> t1 = pml_fetch(g, psi, 1, 0, false, i, j), t2 = pml_fetch(g, psi, 2, 0, false, i, j);
        const T cr = -((rr.M * hx) * rw[RC]) - pml_apply(t1, hz - hzl);
        const T cp = pml_apply(t2, hy - hyl) - (hx - hxd);
        if (MODE == 0) {
            ex = yee::add(lx[0], ex, lx[1], cz);
            ey = yee::add(ly[0], ey, ly[1], cr);
            ez = yee::add(lz[0], ez, lz[1], cp);
        } else {
            ex = yee::half(lx[1], cz);
            ey = yee::half(ly[1], cr);
            ez = yee::half(lz[1], cp);
        }
    } else {
        e_values<T, MODE, CYL>(ex, ey, ez, Hx[c], Hy[c], Hz[c], hxd, hzd, hyl, hzl, lx, ly, lz, rr.M, j,
                               rr.rows + kRowFactors * j);
    }
    if (!CYL && MODE == 0 && aux != nullptr) {
        // Lorentz polarizations of D = eps_inf E + sum P (E slots 0, 1, 2)
        T* ap = aux + (CPLX ? (int64_t)part * 3 * g.n_lor * 2 * g.ncell : 0);
        ex -= yee::lorentz_step(g, ap, 0, c, id_x, lx[0], Ex[c]);
        ey -= yee::lorentz_step(g, ap, 1, c, id_y, ly[0], Ey[c]);
        ez -= yee::lorentz_step(g, ap, 2, c, id_z, lz[0], Ez[c]);
    }
    Ex[c] = ex;
    Ey[c] = ey;
    Ez[c] = ez;
}

template <typename T, int MODE, bool CYL, bool CPLX>
__global__ __launch_bounds__(BX* BY) void k_hred(T* __restrict__ fields, const ChanDev* __restrict__ ch,
                                               const int* __restrict__ slots, Grid2D g,
                                               const T* __restrict__ lut, RedRun<T> rr) {
    const ChanDev d = ch[slots[blockIdx.y]];
    if (MODE == 1 && d.kind != 0) return;   // start: E-kind runs set H^{-1/2}
    const int tiles_x = (g.nx + BX - 1) / BX;
    const int i = (blockIdx.x % tiles_x) * BX + threadIdx.x;
    const int j = (blockIdx.x / tiles_x) * BY + threadIdx.y;
    if (i >= g.nx || j >= g.ny) return;
    T* psi = g.psi ? static_cast<T*>(g.psi) + d.psi_off : nullptr;
    for (int part = 0; part < (CPLX ? 2 : 1); ++part)
        hred_cell<T, MODE, CYL, CPLX>(fields + d.field_off, g, lut, d.kind, rr, i, j, part, psi);
}

template <typename T, int MODE, bool CYL, bool CPLX>
__global__ __launch_bounds__(BX* BY) void k_ered(T* __restrict__ fields, const ChanDev* __restrict__ ch,
                                               const int* __restrict__ slots, Grid2D g,
                                               const T* __restrict__ lut, RedRun<T> rr) {
    const ChanDev d = ch[slots[blockIdx.y]];
    if (MODE == 1 && d.kind != 1) return;   // start: H-kind runs set E^{+1/2}
    const int tiles_x = (g.nx + BX - 1) / BX;
    const int i = (blockIdx.x % tiles_x) * BX + threadIdx.x;
    const int j = (blockIdx.x / tiles_x) * BY + threadIdx.y;
    if (i >= g.nx || j >= g.ny) return;
    T* psi = g.psi ? static_cast<T*>(g.psi) + d.psi_off : nullptr;
    T* aux = g.n_lor > 0 ? static_cast<T*>(g.aux) + d.aux_off : nullptr;
    for (int part = 0; part < (CPLX ? 2 : 1); ++part)
        ered_cell<T, MODE, CYL, CPLX>(fields + d.field_off, g, lut, d.kind, rr, i, j, part, psi, aux);
}

// Every cell of the grid once, block-strided: thread t takes flat cells
// t, t + NTH, ... (consecutive threads on consecutive z).
template <int NTH = kResThreads, typename Body>
__device__ __forceinline__ void for_cells(const Grid2D& g, Body body) {
    const int di = NTH % g.nx, dj = NTH / g.nx;
    int i = threadIdx.x % g.nx, j = threadIdx.x / g.nx;
    while (j < g.ny) {
        body(i, j);
        i += di;
        j += dj;
        if (i >= g.nx) {
            i -= g.nx;
            ++j;
        }
    }
}

// One H (or E) half step of a channel block in global memory by a whole
// block, kBatch cells per thread at a time (4 in FP32, 2 in FP64: the
// register budget of a 1024-thread block): all loads of those cells are
// issued before the first update, then the updates and stores.  Coefficient
// pairs come from Lc, the pairs of the block's kind (6 x 256).
template <typename T>
constexpr int batch_of() {
    return sizeof(T) == 8 ? 2 : 4;
}

template <typename T, int MODE, bool CYL, int NTH = kResThreads, bool CPLX = false>
__device__ __forceinline__ void h_phase(T* __restrict__ F0, const Grid2D& g, const T* __restrict__ Lc,
                                        const RedRun<T>& rr) {
  for (int part = 0; part < (CPLX ? 2 : 1); ++part) {
    T* const F = F0 + (CPLX ? part * 6 * g.ncell : 0);
    const T* const Fo = F0 + (CPLX ? (1 - part) * 6 * g.ncell : 0);   // the other part (complex runs)
    constexpr int kBatch = batch_of<T>();
    const T* Ex = F;
    const T* Ey = F + g.ncell;
    const T* Ez = F + 2 * g.ncell;
    T* Hx = F + 3 * g.ncell;
    T* Hy = F + 4 * g.ncell;
    T* Hz = F + 5 * g.ncell;
    const int nx = g.nx, ny = g.ny;
    const int di = NTH % nx, dj = NTH / nx;
    int i = threadIdx.x % nx, j = threadIdx.x / nx;
    while (j < ny) {
        T ex[kBatch], ey[kBatch], ez[kBatch], ezu[kBatch], exu[kBatch], ezr[kBatch], eyr[kBatch];
        T hx[kBatch], hy[kBatch], hz[kBatch];
        int cc[kBatch], jj[kBatch];
        uint32_t id[kBatch];
#pragma unroll
        for (int q = 0; q < kBatch; ++q) {
            jj[q] = j;
            cc[q] = j * nx + i;
            if (j < ny) {
                const int c = cc[q];
                const bool in_r = i + 1 < nx, in_u = j + 1 < ny;
                const int cu = in_u ? c + nx : i;
                const bool has_u = in_u || (!CYL && g.pery);   // the tube wall is never periodic
                ezu[q] = has_u ? Ez[cu] : T(0);
                exu[q] = has_u ? Ex[cu] : T(0);
                if (in_r) {
                    ezr[q] = Ez[c + 1];
                    eyr[q] = Ey[c + 1];
                } else if (!g.perx) {
                    ezr[q] = eyr[q] = T(0);
                } else if (CPLX) {
                    const int w = c + 1 - nx;
                    ezr[q] = bloch_fwd(Ez[w], Fo[2 * (int)g.ncell + w], part, rr.pc, rr.ps);
                    eyr[q] = bloch_fwd(Ey[w], Fo[(int)g.ncell + w], part, rr.pc, rr.ps);
                } else {
                    ezr[q] = Ez[c + 1 - nx];
                    eyr[q] = Ey[c + 1 - nx];
                }
                ex[q] = Ex[c];
                ey[q] = Ey[c];
                ez[q] = Ez[c];
                hx[q] = Hx[c];
                hy[q] = Hy[c];
                hz[q] = Hz[c];
                id[q] = uint32_t(g.ids[CF_HX][c]) | (uint32_t(g.ids[CF_HY][c]) << 8) |
                        (uint32_t(g.ids[CF_HZ][c]) << 16);
            }
            i += di;
            j += dj;
            if (i >= nx) {
                i -= nx;
                ++j;
            }
        }
#pragma unroll
        for (int q = 0; q < kBatch; ++q) {
            if (jj[q] < ny) {
                const int c = cc[q];
                h_values<T, MODE, CYL>(hx[q], hy[q], hz[q], ex[q], ey[q], ez[q], ezu[q], exu[q], ezr[q], eyr[q],
                                  Lc + ((CF_HX << 8) + (int)(id[q] & 255)) * 2,
                                  Lc + ((CF_HY << 8) + (int)((id[q] >> 8) & 255)) * 2,
                                  Lc + ((CF_HZ << 8) + (int)(id[q] >> 16)) * 2, rr.M, jj[q],
                                  rr.rows + kRowFactors * jj[q]);
                Hx[c] = hx[q];
                Hy[c] = hy[q];
                Hz[c] = hz[q];
            }
        }
    }
  }
}

template <typename T, int MODE, bool CYL, int NTH = kResThreads, bool CPLX = false>
__device__ __forceinline__ void e_phase(T* __restrict__ F0, const Grid2D& g, const T* __restrict__ Lc,
                                        const RedRun<T>& rr) {
  for (int part = 0; part < (CPLX ? 2 : 1); ++part) {
    T* const F = F0 + (CPLX ? part * 6 * g.ncell : 0);
    const T* const Fo = F0 + (CPLX ? (1 - part) * 6 * g.ncell : 0);
    constexpr int kBatch = batch_of<T>();
    T* Ex = F;
    T* Ey = F + g.ncell;
    T* Ez = F + 2 * g.ncell;
    const T* Hx = F + 3 * g.ncell;
    const T* Hy = F + 4 * g.ncell;
    const T* Hz = F + 5 * g.ncell;
    const int nx = g.nx, ny = g.ny;
    const int di = NTH % nx, dj = NTH / nx;
    int i = threadIdx.x % nx, j = threadIdx.x / nx;
    while (j < ny) {
        T hx[kBatch], hy[kBatch], hz[kBatch], hxd[kBatch], hzd[kBatch], hyl[kBatch], hzl[kBatch];
        T ex[kBatch], ey[kBatch], ez[kBatch];
        int cc[kBatch], jj[kBatch];
        uint32_t id[kBatch];
#pragma unroll
        for (int q = 0; q < kBatch; ++q) {
            jj[q] = j;
            cc[q] = j * nx + i;
            if (j < ny) {
                const int c = cc[q];
                const bool in_d = j > 0;
                const int cd = in_d ? c - nx : c + (int)g.ncell - nx;
                const bool has_d = in_d || (!CYL && g.pery);
                hxd[q] = has_d ? Hx[cd] : T(0);
                hzd[q] = has_d ? Hz[cd] : T(0);
                if (i > 0) {
                    hyl[q] = Hy[c - 1];
                    hzl[q] = Hz[c - 1];
                } else if (!g.perx) {
                    hyl[q] = hzl[q] = T(0);
                } else if (CPLX) {
                    const int w = c - 1 + nx;
                    hyl[q] = bloch_bwd(Hy[w], Fo[4 * (int)g.ncell + w], part, rr.pc, rr.ps);
                    hzl[q] = bloch_bwd(Hz[w], Fo[5 * (int)g.ncell + w], part, rr.pc, rr.ps);
                } else {
                    hyl[q] = Hy[c - 1 + nx];
                    hzl[q] = Hz[c - 1 + nx];
                }
                hx[q] = Hx[c];
                hy[q] = Hy[c];
                hz[q] = Hz[c];
                ex[q] = Ex[c];
                ey[q] = Ey[c];
                ez[q] = Ez[c];
                id[q] = uint32_t(g.ids[CF_EX][c]) | (uint32_t(g.ids[CF_EY][c]) << 8) |
                        (uint32_t(g.ids[CF_EZ][c]) << 16);
            }
            i += di;
            j += dj;
            if (i >= nx) {
                i -= nx;
                ++j;
            }
        }
#pragma unroll
        for (int q = 0; q < kBatch; ++q) {
            if (jj[q] < ny) {
                const int c = cc[q];
                e_values<T, MODE, CYL>(ex[q], ey[q], ez[q], hx[q], hy[q], hz[q], hxd[q], hzd[q], hyl[q], hzl[q],
                                  Lc + ((CF_EX << 8) + (int)(id[q] & 255)) * 2,
                                  Lc + ((CF_EY << 8) + (int)((id[q] >> 8) & 255)) * 2,
                                  Lc + ((CF_EZ << 8) + (int)(id[q] >> 16)) * 2, rr.M, jj[q],
                                  rr.rows + kRowFactors * jj[q]);
                Ex[c] = ex[q];
                Ey[c] = ey[q];
                Ez[c] = ez[q];
            }
        }
    }
  }
}

template <typename T, bool CYL, bool CPLX>
__global__ __launch_bounds__(kResThreads) void k_red_resident(T* __restrict__ fields, const ChanDev* __restrict__ ch,
                                                              const int* __restrict__ slots, Grid2D g, RedOrders ord,
                                                              RedSpan sp, SurfTables t, double dA, double* __restrict__ acc,
                                                              double* __restrict__ gamma, int gamma_stride) {
    __shared__ double red[yee::kSurfThreads / 64];
    __shared__ T Lc[6 * 256 * 2];
    const int slot = slots[blockIdx.x];
    const ChanDev d = ch[slot];
    const int m = d.order;
    const T* lut = static_cast<const T*>(ord.lut) + m * ord.lut_stride;
    const double* ktab = ord.ktab + m * ord.ktab_stride;
    const int s0 = sp.s0[m], s1 = sp.s1[m];
    const double dt = ord.dt[m];
    T* F = fields + d.field_off;
    const T* lk = lut + d.kind * 6 * 256 * 2;
    for (int k = threadIdx.x; k < 6 * 256 * 2; k += kResThreads) Lc[k] = lk[k];
    const RedRun<T> rr{T(ord.coup[m]), static_cast<const T*>(ord.rows), T(ord.ph_c[m]), T(ord.ph_s[m])};
    if (s0 == 0) {   // first part of the run: clear, kick and start
        const int64_t nval = (CPLX ? 12 : 6) * g.ncell;
        for (int64_t k = threadIdx.x; k < nval; k += kResThreads) F[k] = T(0);
        __syncthreads();
        // kick: the source component's surface deposit (one writer per point)
        for (int u = threadIdx.x; u < d.n_uniq; u += kResThreads) {
            const int k0 = t.uoff[d.u_off + u], k1 = t.uoff[d.u_off + u + 1];
            double s = 0.0;
            for (int k = k0; k < k1; ++k) s += t.uw[k] * t.basis[d.basis_off + t.usamp[k]];
            fields[d.src_off + t.uidx[d.u_off + u]] = T(d.kick_scale * s);
        }
        __syncthreads();
        if (d.kind == 0) h_phase<T, 1, CYL, kResThreads, CPLX>(F, g, Lc, rr);
        else e_phase<T, 1, CYL, kResThreads, CPLX>(F, g, Lc, rr);
    }
    __syncthreads();
    const T* X = fields + d.meas_off;
    double sum = 0.0, comp = 0.0;
    if (threadIdx.x == 0) {
        sum = acc[2 * slot];
        comp = acc[2 * slot + 1];
    }
    for (int step = s0; step < s1; ++step) {
        h_phase<T, 0, CYL, kResThreads, CPLX>(F, g, Lc, rr);
        __syncthreads();
        e_phase<T, 0, CYL, kResThreads, CPLX>(F, g, Lc, rr);
        __syncthreads();
        // every read of X ends at the barrier inside; the next writes of the
        // fields come after it
        const double s = yee::block_surface_sum(d, t, [&](int32_t idx) { return (double)X[idx]; }, red);
        if (threadIdx.x == 0) {
            const double G = dA * s;
            yee::neumaier(sum, comp, (dt * ktab[step]) * G);
            if (gamma) gamma[(int64_t)step * gamma_stride + slot] = G;
        }
    }
    if (threadIdx.x == 0) {
        acc[2 * slot] = sum;
        acc[2 * slot + 1] = comp;
    }
}

// Length of the exchange array of the register kernel: 3 n values per part
// (np = 2 for complex runs), and at least the 6 x 256 coefficient pairs it
// holds during the start.
__host__ __device__ constexpr int regs_x_len(int n, int np) {
    return 3 * np * n > 6 * 256 * 2 ? 3 * np * n : 6 * 256 * 2;
}

// Register-resident solve: the clear, kick and start as in k_red_resident,
// then every thread keeps the six fields of its K cells (flat cells t,
// t + NTH, ...) in registers for all steps.  LDS holds one array of 3 x ncell
// values that carries the E triple during the H half step and the H triple
// during the E half step (the neighbour exchange), the six material ids of
// every cell packed in 4 bits each (ord.idw; 15 stands for the wall id), and
// the 6 x 16 coefficient pairs of the block's kind.  The surface projection
// reads the measured component from the exchange array (H components before
// the E half step overwrites it: the values the other drivers read after the
// step).  A cell's coordinates are recomputed in every half step from the
// thread's first cell, passed through an empty asm statement so that the
// compiler keeps no per-cell addresses in registers across steps.
// CPLX (Bloch-periodic x): both parts of every field in registers, the
// exchange array holds the real part's triple and then the imaginary part's,
// and the neighbours across the periodic x edge take the Bloch phase as in
// the other drivers; the surface reads the real part.
template <typename T, int K, int NTH, bool CYL, bool CPLX>
__global__ __launch_bounds__(NTH) void k_red_regs(T* __restrict__ fields, const ChanDev* __restrict__ ch,
                                                  const int* __restrict__ slots, Grid2D g, RedOrders ord,
                                                  RedSpan sp, SurfTables t, double dA, double* __restrict__ acc,
                                                  double* __restrict__ gamma, int gamma_stride) {
    constexpr int NP = CPLX ? 2 : 1;               // parts: real (and imaginary)
    extern __shared__ double lds_dyn[];
    __shared__ double red[yee::kSurfThreads / 64];   // wave partials of the pending measurement
    const int n = (int)g.ncell;
    T* X = reinterpret_cast<T*>(lds_dyn);          // 3 n exchange values per part
    T* Lg = X;                                      // the kind's full table, for the start (before X is used)
    T* Lc = X + regs_x_len(n, NP);                  // 6 x 16 (a, b) pairs
    T* R = Lc + 6 * 16 * 2;                         // row factors (kRowFactors per row)
    uint32_t* W = reinterpret_cast<uint32_t*>(R + kRowFactors * g.ny);   // packed ids per cell
    const int slot = slots[blockIdx.x];
    const ChanDev d = ch[slot];
    const int m = d.order;
    const T* lut = static_cast<const T*>(ord.lut) + m * ord.lut_stride;
    const double* ktab = ord.ktab + m * ord.ktab_stride;
    const int s0 = sp.s0[m], s1 = sp.s1[m];
    const bool resume_later = s1 < ord.steps[m];
    const double dt = ord.dt[m];
    T* F = fields + d.field_off;
    const T* lk = lut + d.kind * 6 * 256 * 2;
    if (s0 == 0)
        for (int k = threadIdx.x; k < 6 * 256 * 2; k += NTH) Lg[k] = lk[k];
    for (int k = threadIdx.x; k < 6 * 16 * 2; k += NTH) {
        const int cmp = k / 32, q = (k / 2) % 16;
        Lc[k] = lk[((cmp << 8) + (q == 15 ? 255 : q)) * 2 + (k & 1)];
    }
    for (int k = threadIdx.x; k < n; k += NTH) W[k] = ord.idw[k];
    for (int k = threadIdx.x; k < kRowFactors * g.ny; k += NTH) R[k] = static_cast<const T*>(ord.rows)[k];
    const RedRun<T> rr{T(ord.coup[m]), R, CPLX ? T(ord.ph_c[m]) : T(1), CPLX ? T(ord.ph_s[m]) : T(0)};
    if (s0 == 0) {   // first part of the run: clear, kick and start
        for (int64_t k = threadIdx.x; k < NP * 6 * g.ncell; k += NTH) F[k] = T(0);
        __syncthreads();
        // (the exchange array takes over Lg's space after the start)
        for (int u = threadIdx.x; u < d.n_uniq; u += NTH) {
            const int k0 = t.uoff[d.u_off + u], k1 = t.uoff[d.u_off + u + 1];
            double s = 0.0;
            for (int k = k0; k < k1; ++k) s += t.uw[k] * t.basis[d.basis_off + t.usamp[k]];
            fields[d.src_off + t.uidx[d.u_off + u]] = T(d.kick_scale * s);
        }
        __syncthreads();
        if (d.kind == 0) h_phase<T, 1, CYL, NTH, CPLX>(F, g, Lg, rr);
        else e_phase<T, 1, CYL, NTH, CPLX>(F, g, Lg, rr);
    }
    __syncthreads();
    T e0[NP][K], e1[NP][K], e2[NP][K], h0[NP][K], h1[NP][K], h2[NP][K];
#pragma unroll
    for (int p = 0; p < NP; ++p)
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const int c = threadIdx.x + k * NTH;
            const T* Fp = F + p * 6 * n;
            T* Xp = X + p * 3 * n;
            if (c < n) {
                e0[p][k] = Fp[c];
                e1[p][k] = Fp[n + c];
                e2[p][k] = Fp[2 * n + c];
                h0[p][k] = Fp[3 * n + c];
                h1[p][k] = Fp[4 * n + c];
                h2[p][k] = Fp[5 * n + c];
                Xp[c] = e0[p][k];
                Xp[n + c] = e1[p][k];
                Xp[2 * n + c] = e2[p][k];
            } else {
                e0[p][k] = e1[p][k] = e2[p][k] = h0[p][k] = h1[p][k] = h2[p][k] = T(0);
            }
        }
    __syncthreads();
    const bool meas_h = d.meas_slot >= 3;
    const T* Xq = X + (d.meas_slot % 3) * n;
    const int nx = g.nx, ny = g.ny;
    const int di = NTH % nx, dj = NTH / nx;
    int i0 = threadIdx.x % nx, j0 = threadIdx.x / nx;
    double sum = 0.0, comp = 0.0;
    if (threadIdx.x == 0) {
        sum = acc[2 * slot];
        comp = acc[2 * slot + 1];
    }
    auto pair = [&](int cmp, uint32_t w) { return Lc + ((cmp << 4) + (int)((w >> (4 * cmp)) & 15)) * 2; };
    // The surface sum of a step is split: its wave partials are formed right
    // after the exchange array holds the measured fields, with no barrier of
    // their own, and thread 0 adds them up behind the next barrier of the
    // half steps.  One partial buffer suffices: thread 0 reads it before the
    // barrier after that, and the next partials are written later still.
    int pending = -1;                    // step whose partials wait in red
    auto measure = [&](int step) {
        yee::wave_surface_partials(d, t, [&](int32_t idx) { return (double)Xq[idx]; }, red);
        pending = step;
    };
    auto finish = [&]() {               // call right after a barrier
        if (pending >= 0 && threadIdx.x == 0) {
            const double G = dA * yee::wave_partials_total(red);
            yee::neumaier(sum, comp, (dt * ktab[pending]) * G);
            if (gamma) gamma[(int64_t)pending * gamma_stride + slot] = G;
        }
        pending = -1;
    };
    for (int step = s0; step < s1; ++step) {
        asm volatile("" : "+v"(i0), "+v"(j0));
        {
            int i = i0, j = j0;
#pragma unroll
            for (int k = 0; k < K; ++k) {
                if (j < ny) {
                    const int c = j * nx + i;
                    const bool in_r = i + 1 < nx, in_u = j + 1 < ny;
                    const uint32_t w = W[c];
                    const int cu = in_u ? c + nx : i;
                    const bool has_u = in_u || (!CYL && g.pery);   // the tube wall is never periodic
#pragma unroll
                    for (int p = 0; p < NP; ++p) {
                        const T* Xp = X + p * 3 * n;
                        const T ezu = has_u ? Xp[2 * n + cu] : T(0);
                        const T exu = has_u ? Xp[cu] : T(0);
                        T ezr, eyr;
                        if (in_r || !g.perx || !CPLX) {
                            ezr = in_r ? Xp[2 * n + c + 1] : (g.perx ? Xp[2 * n + c + 1 - nx] : T(0));
                            eyr = in_r ? Xp[n + c + 1] : (g.perx ? Xp[n + c + 1 - nx] : T(0));
                        } else {   // across the Bloch-periodic edge
                            const T* Xo = X + (1 - p) * 3 * n;
                            const int wr = c + 1 - nx;
                            ezr = bloch_fwd(Xp[2 * n + wr], Xo[2 * n + wr], p, rr.pc, rr.ps);
                            eyr = bloch_fwd(Xp[n + wr], Xo[n + wr], p, rr.pc, rr.ps);
                        }
                        h_values<T, 0, CYL>(h0[p][k], h1[p][k], h2[p][k], e0[p][k], e1[p][k], e2[p][k], ezu, exu,
                                            ezr, eyr, pair(CF_HX, w), pair(CF_HY, w), pair(CF_HZ, w), rr.M, j,
                                            R + kRowFactors * j);
                    }
                }
                i += di;
                j += dj;
                if (i >= nx) {
                    i -= nx;
                    ++j;
                }
            }
        }
        __syncthreads();
        finish();
#pragma unroll
        for (int p = 0; p < NP; ++p)
#pragma unroll
            for (int k = 0; k < K; ++k) {
                const int c = threadIdx.x + k * NTH;
                if (c < n) {
                    X[p * 3 * n + c] = h0[p][k];
                    X[p * 3 * n + n + c] = h1[p][k];
                    X[p * 3 * n + 2 * n + c] = h2[p][k];
                }
            }
        __syncthreads();
        if (meas_h) measure(step);
        asm volatile("" : "+v"(i0), "+v"(j0));
        {
            int i = i0, j = j0;
#pragma unroll
            for (int k = 0; k < K; ++k) {
                if (j < ny) {
                    const int c = j * nx + i;
                    const bool in_d = j > 0;
                    const uint32_t w = W[c];
                    const int cd = in_d ? c - nx : c + n - nx;
                    const bool has_d = in_d || (!CYL && g.pery);
#pragma unroll
                    for (int p = 0; p < NP; ++p) {
                        const T* Xp = X + p * 3 * n;
                        const T hxd = has_d ? Xp[cd] : T(0);
                        const T hzd = has_d ? Xp[2 * n + cd] : T(0);
                        T hyl, hzl;
                        if (i > 0 || !g.perx || !CPLX) {
                            hyl = i > 0 ? Xp[n + c - 1] : (g.perx ? Xp[n + c - 1 + nx] : T(0));
                            hzl = i > 0 ? Xp[2 * n + c - 1] : (g.perx ? Xp[2 * n + c - 1 + nx] : T(0));
                        } else {   // across the Bloch-periodic edge
                            const T* Xo = X + (1 - p) * 3 * n;
                            const int wl = c - 1 + nx;
                            hyl = bloch_bwd(Xp[n + wl], Xo[n + wl], p, rr.pc, rr.ps);
                            hzl = bloch_bwd(Xp[2 * n + wl], Xo[2 * n + wl], p, rr.pc, rr.ps);
                        }
                        e_values<T, 0, CYL>(e0[p][k], e1[p][k], e2[p][k], h0[p][k], h1[p][k], h2[p][k], hxd, hzd,
                                            hyl, hzl, pair(CF_EX, w), pair(CF_EY, w), pair(CF_EZ, w), rr.M, j,
                                            R + kRowFactors * j);
                    }
                }
                i += di;
                j += dj;
                if (i >= nx) {
                    i -= nx;
                    ++j;
                }
            }
        }
        __syncthreads();
        finish();
#pragma unroll
        for (int p = 0; p < NP; ++p)
#pragma unroll
            for (int k = 0; k < K; ++k) {
                const int c = threadIdx.x + k * NTH;
                if (c < n) {
                    X[p * 3 * n + c] = e0[p][k];
                    X[p * 3 * n + n + c] = e1[p][k];
                    X[p * 3 * n + 2 * n + c] = e2[p][k];
                }
            }
        __syncthreads();
        if (!meas_h) measure(step);
    }
    __syncthreads();
    finish();
    if (threadIdx.x == 0) {
        acc[2 * slot] = sum;
        acc[2 * slot + 1] = comp;
    }
    if (resume_later) {   // a later launch resumes from memory
        // the thread index and the block's field pointer are formed again
        // here (through an empty asm statement) rather than kept live
        // through the step loop
        int tid = threadIdx.x;
        asm volatile("" : "+v"(tid));
        T* Fe = fields + ch[slots[blockIdx.x]].field_off;
#pragma unroll
        for (int p = 0; p < NP; ++p)
#pragma unroll
            for (int k = 0; k < K; ++k) {
                const int c = tid + k * NTH;
                T* Fp = Fe + p * 6 * n;
                if (c < n) {
                    Fp[c] = e0[p][k];
                    Fp[n + c] = e1[p][k];
                    Fp[2 * n + c] = e2[p][k];
                    Fp[3 * n + c] = h0[p][k];
                    Fp[4 * n + c] = h1[p][k];
                    Fp[5 * n + c] = h2[p][k];
                }
            }
    }
}

template <typename T>
size_t regs_lds_bytes(const Grid2D& g, int np) {
    return ((size_t)regs_x_len((int)g.ncell, np) + 6 * 16 * 2 + kRowFactors * (size_t)g.ny) * sizeof(T) +
           4 * (size_t)g.ncell;
}


// Register variants (cells per thread K, threads per block NTH), each
// without register spills, smallest first: FP32 up to 10240 cells, FP64 up
// to 6144 (the LDS of a CU, 16 or 28 bytes per cell, bounds both first).
struct RegVariant {
    int K, NTH;
};
constexpr int kNumRegVariants = 6;
template <typename T>
constexpr RegVariant kRegVariants[kNumRegVariants] = {{1, 1024}, {2, 1024}, {4, 1024}, {6, 1024}, {8, 1024}, {10, 1024}};
template <>
constexpr RegVariant kRegVariants<double>[kNumRegVariants] = {{1, 1024}, {2, 1024}, {3, 1024}, {4, 1024}, {6, 1024},
                                                               {6, 1024}};

// LDS bytes a block may take on the current device
inline size_t device_lds_limit() {
    int dev = 0, v = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 65536;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess) return 65536;
    return (size_t)v;
}

// Dynamic LDS above 64 KB needs the kernel's attribute raised first.  The
// attribute is a cap and is only ever raised (under a lock), so solves on
// concurrent host threads never lower it below what another one launches
// with; false when the runtime refuses (the caller then takes the
// global-memory variant).
template <typename T, int K, int NTH, bool CYL, bool CPLX>
bool regs_lds_ok(size_t lds) {
    if (lds <= 65536) return true;
    static std::mutex mu;
    static size_t cap = 65536;
    std::lock_guard<std::mutex> lk(mu);
    if (lds <= cap) return true;
    const hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_red_regs<T, K, NTH, CYL, CPLX>),
                                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    cap = lds;
    return true;
}

// Register variants a complex run may take (both parts of every field in
// registers): the first kCplxRegVariants, which do not spill (FP32 up to 6
// cells per thread, FP64 up to 3).
template <typename T>
constexpr int kCplxRegVariants = 4;
template <>
constexpr int kCplxRegVariants<double> = 3;

// Launch register variant v if the grid fits it: *launched tells whether it did.
template <typename T, int V, bool CYL, bool CPLX>
hipError_t regs_try(int64_t ncell, size_t lds, bool* launched, T* fields, const ChanDev* ch, const int* slots,
                    int nslots, const Grid2D& g, const RedOrders& ord, const RedSpan& sp, const SurfTables& t,
                    double dA, double* acc, double* gamma, int gamma_stride, hipStream_t s) {
    *launched = false;
    if constexpr (CPLX && V >= kCplxRegVariants<T>) {
        return hipSuccess;
    } else {
        constexpr int K = kRegVariants<T>[V].K, NTH = kRegVariants<T>[V].NTH;
        if (ncell > (int64_t)K * NTH || !regs_lds_ok<T, K, NTH, CYL, CPLX>(lds)) return hipSuccess;
        *launched = true;
        hipLaunchKernelGGL((k_red_regs<T, K, NTH, CYL, CPLX>), dim3(nslots), dim3(NTH), lds, s, fields, ch, slots, g,
                           ord, sp, t, dA, acc, gamma, gamma_stride);
        return hipGetLastError();
    }
}

}  // namespace

template <typename T>
hipError_t launch_hred(int mode, double coupling, int axis, T* fields, const ChanDev* ch, const int* slots,
                       int nslots, const Grid2D& g, const T* lut, const T* rows, double ph_c, double ph_s, int cplx,
                       hipStream_t s) {
    if (nslots <= 0) return hipSuccess;
    const dim3 grid = grid_red(g, nslots), block(BX, BY, 1);
    const RedRun<T> rr{T(coupling), rows, T(ph_c), T(ph_s)};
#define CF_HCYL(M, C, X) hipLaunchKernelGGL((k_hred<T, M, C, X>), grid, block, 0, s, fields, ch, slots, g, lut, rr)
    if (axis) {
        if (mode == 0) CF_HCYL(0, true, false);
        else CF_HCYL(1, true, false);
    } else if (cplx) {
        if (mode == 0) CF_HCYL(0, false, true);
        else CF_HCYL(1, false, true);
    } else {
        if (mode == 0) CF_HCYL(0, false, false);
        else CF_HCYL(1, false, false);
    }
#undef CF_HCYL
    return hipGetLastError();
}

template <typename T>
hipError_t launch_ered(int mode, double coupling, int axis, T* fields, const ChanDev* ch, const int* slots,
                       int nslots, const Grid2D& g, const T* lut, const T* rows, double ph_c, double ph_s, int cplx,
                       hipStream_t s) {
    if (nslots <= 0) return hipSuccess;
    const dim3 grid = grid_red(g, nslots), block(BX, BY, 1);
    const RedRun<T> rr{T(coupling), rows, T(ph_c), T(ph_s)};
#define CF_ECYL(M, C, X) hipLaunchKernelGGL((k_ered<T, M, C, X>), grid, block, 0, s, fields, ch, slots, g, lut, rr)
    if (axis) {
        if (mode == 0) CF_ECYL(0, true, false);
        else CF_ECYL(1, true, false);
    } else if (cplx) {
        if (mode == 0) CF_ECYL(0, false, true);
        else CF_ECYL(1, false, true);
    } else {
        if (mode == 0) CF_ECYL(0, false, false);
        else CF_ECYL(1, false, false);
    }
#undef CF_ECYL
    return hipGetLastError();
}

template <typename T, bool CYL, bool CPLX>
hipError_t resident_launch(int variant, T* fields, const ChanDev* ch, const int* slots, int nslots,
                           const Grid2D& g, const RedOrders& ord, const RedSpan& sp, const SurfTables& t, double dA,
                           double* acc, double* gamma, int gamma_stride, hipStream_t s, int* used) {
    *used = 0;
    if (nslots <= 0) return hipSuccess;
    const size_t dyn = regs_lds_bytes<T>(g, CPLX ? 2 : 1);
    if (variant != 2 && ord.idw && dyn + 64 <= device_lds_limit()) {
        bool launched = false;
        hipError_t e = hipSuccess;
        auto attempt = [&](auto v) {
            if (!launched && e == hipSuccess)
                e = regs_try<T, decltype(v)::value, CYL, CPLX>(g.ncell, dyn, &launched, fields, ch, slots, nslots, g,
                                                               ord, sp, t, dA, acc, gamma, gamma_stride, s);
        };
        attempt(std::integral_constant<int, 0>{});
        attempt(std::integral_constant<int, 1>{});
        attempt(std::integral_constant<int, 2>{});
        attempt(std::integral_constant<int, 3>{});
        attempt(std::integral_constant<int, 4>{});
        attempt(std::integral_constant<int, 5>{});
        static_assert(kNumRegVariants == 6, "one attempt per register variant");
        if (e != hipSuccess) return e;
        if (launched) {
            *used = 1;
            return hipSuccess;
        }
    }
    *used = 2;
    hipLaunchKernelGGL((k_red_resident<T, CYL, CPLX>), dim3(nslots), dim3(kResThreads), 0, s, fields, ch, slots, g, ord, sp,
                       t, dA, acc, gamma, gamma_stride);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_red_resident_span(int variant, T* fields, const ChanDev* ch, const int* slots, int nslots,
                                    const Grid2D& g, const RedOrders& ord, const RedSpan& sp, const SurfTables& t,
                                    double dA, double* acc, double* gamma, int gamma_stride, hipStream_t s,
                                    int* used) {
    if (ord.axis)
        return resident_launch<T, true, false>(variant, fields, ch, slots, nslots, g, ord, sp, t, dA, acc, gamma,
                                               gamma_stride, s, used);
    if (ord.cplx)
        return resident_launch<T, false, true>(variant, fields, ch, slots, nslots, g, ord, sp, t, dA, acc, gamma,
                                               gamma_stride, s, used);
    return resident_launch<T, false, false>(variant, fields, ch, slots, nslots, g, ord, sp, t, dA, acc, gamma,
                                            gamma_stride, s, used);
}

template <typename T>
hipError_t launch_red_resident(int variant, T* fields, const ChanDev* ch, const int* slots, int nslots,
                               const Grid2D& g, const RedOrders& ord, const SurfTables& t, double dA, double* acc,
                               double* gamma, int gamma_stride, hipStream_t s, int* used) {
    RedSpan sp{};
    for (int m = 0; m < kMaxOrders; ++m) sp.s1[m] = ord.steps[m];
    return launch_red_resident_span<T>(variant, fields, ch, slots, nslots, g, ord, sp, t, dA, acc, gamma,
                                       gamma_stride, s, used);
}

#define CF_RED_INSTANTIATE(T)                                                                                   \
    template hipError_t launch_hred<T>(int, double, int, T*, const ChanDev*, const int*, int, const Grid2D&,  \
                                       const T*, const T*, double, double, int, hipStream_t);                  \
    template hipError_t launch_ered<T>(int, double, int, T*, const ChanDev*, const int*, int, const Grid2D&,  \
                                       const T*, const T*, double, double, int, hipStream_t);                  \
    template hipError_t launch_red_resident<T>(int, T*, const ChanDev*, const int*, int, const Grid2D&,       \
                                               const RedOrders&, const SurfTables&, double, double*, double*, \
                                               int, hipStream_t, int*);                                         \
    template hipError_t launch_red_resident_span<T>(int, T*, const ChanDev*, const int*, int, const Grid2D&,  \
                                                    const RedOrders&, const RedSpan&, const SurfTables&, double, \
                                                    double*, double*, int, hipStream_t, int*);
CF_RED_INSTANTIATE(float)
CF_RED_INSTANTIATE(double)
#undef CF_RED_INSTANTIATE

}  // namespace cf
