// Device-side tables and kernel launchers shared by the HIP sources and the
// C ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace cf {

// Per-channel descriptor on the device.  Offsets are element offsets into
// the field array (fields), the gather tables (gidx/gw), the scatter tables
// (uidx/uoff) and the basis table.
struct ChanDev {
    int64_t field_off;   // first element of the channel's field block
    int64_t psi_off;     // first element of the channel's CPML block (3D; 2D split kernels)
    int32_t inst;        // instance of a fused launch
    int32_t pol;         // CF_POL_TM / CF_POL_TE / CF_POL_3D
    int32_t local;       // channel index within its instance (accumulator, Gamma column)
    int32_t order;       // azimuthal order m (cylindrical problems)
    int64_t src_off;     // field_off + slot(src) * ncell
    int64_t meas_off;    // field_off + slot(meas) * ncell
    int32_t kind;        // 0 E-current source, 1 H-current source
    int32_t nsamp;       // samples on the channel's face
    int32_t P;           // interpolation points per sample of the measured component
    int32_t g_off;       // gather table offset (measured component), entries = nsamp*P
    int32_t u_off;       // scatter table: first distinct point (source component)
    int32_t n_uniq;      // number of distinct source points
    int32_t basis_off;   // first basis value of the channel's row
    int32_t meas_slot;   // slot of the measured component in the field block
    double kick_scale;   // -res / (eps_S or mu_S)
    int64_t aux_off;     // first element of the channel's polarization block (dispersive media)
};

// Material id of cells outside a non-periodic grid inside a fused tile's
// halo: every coefficient table maps it to a = b = 0.
constexpr int kNullId = 254;

// Grid and table pointers of one launch.
struct Grid2D {
    int nx, ny;
    int64_t ncell;
    int perx, pery;
    const uint8_t* ids[6];   // per-component material ids
    // Dispersive media (split E half step): per material id a row of
    // kLorStride(n_lor) doubles [flag, 1/eps_inf, (c1, c2, c3) per term] with
    // P^{m+1} = c1 P^m - c2 P^{m-1} + c3 E^m; flag != 0 marks an id with terms.
    // aux holds per channel (at ChanDev.aux_off) per E slot e and term j the
    // pair (P^m, P^{m-1}) as two grids: aux[((e * n_lor + j) * 2 + k) * ncell + cell].
    int n_lor;
    const double* lor;
    void* aux;
    // CPML along x (axis 0) and y (axis 1), split kernels only: pml[a]
    // layers at each end of axis a (0: none).  pml_tab[a] holds 4 rows of
    // n_a values: b and c at the half-cell positions (H components), then b
    // and c at the integer positions (E components).  psi (field precision,
    // the channel's block at ChanDev.psi_off) holds per part (complex runs:
    // real, imaginary) and per field slot s an x array of ny * 2 pml[0]
    // values and a y array of 2 pml[1] * nx values; psi_slot is their sum.
    int pml[2];
    const double* pml_tab[2];
    void* psi;
    int64_t psi_slot;
};
constexpr int kLorStride(int n_lor) { return 2 + 3 * n_lor; }

struct SurfTables {
    const int32_t* gidx;
    const double* gw;
    const int32_t* uidx;
    const int32_t* uoff;     // CSR offsets, global
    const int32_t* usamp;    // global sample index into the basis row
    const double* uw;
    const double* basis;
};

// One problem instance of a fused (2D) launch.  Several instances with
// different grids, materials and surfaces can share one launch; each has its
// own time origin `start` on the launch clock and its own step count.
struct InstDev {
    void* fa;              // field buffers of this instance (ping-pong): a launch
    void* fb;              // with parity 0 reads fa and writes fb, parity 1 the reverse
    double* acc;           // (sum, compensation) per channel, indexed by ChanDev.local
    int nx, ny;
    int64_t ncell;
    int perx, pery;
    const uint8_t* ids[6];
    const void* lut;       // coefficient table (field precision)
    int base_x, base_y;    // first cell of tile 0 (<= 0)
    int ntx, nty;          // tiles per axis
    int stile;             // tile (ty * ntx + tx) holding every surface stencil point
    int start;             // launch-clock step at which this instance's step 0 runs
    int nsteps;            // time steps of this instance
    int pad;
    double dt, dA;
    const double* ktab;    // K(t_m) of this instance
    double* gamma;         // optional Gamma rows (stride gamma_stride, column = ChanDev.local)
    int64_t gamma_stride;
    SurfTables t;          // surface tables the instance's channel offsets refer to
};

// Work item of a fused launch: channel descriptor `slot`, tile `tile` of its
// instance, and the tile's live waves.  slot < 0 is padding.
struct WorkItem {
    int slot, tile;
    uint32_t waves;   // bit w: wave w of the tile has a cell that can change (the host's plan)
};

// Tile interior (tx x ty cells), halo / maximum steps per launch and rows
// per wave (b) of the fused kernel's variants (index = variant); the region
// a block holds is (tx + 2 kh) x (ty + 2 kh) cells in (ty + 2 kh) / b waves.
struct TBShape {
    int tx, ty, kh, b;
};
constexpr int kMaxVariants = 16;
template <typename T>
int tb_variants(TBShape* out, int max);

// 3D launch geometry.  The CPML along z has `pml` layers at each end; the
// psi block of a channel is 4 components (Hx dz Ey, Hy dz Ex, Ex dz Hy,
// Ey dz Hx) of psi_comp = 2 * pml * ny * nx values each.  pml_bh/pml_ch
// (pml_be/pml_ce) hold b and c at the z positions of H_x, H_y (E_x, E_y).
struct Grid3D {
    int nx, ny, nz;
    int64_t ncell;
    int per[3];
    const uint8_t* ids[6];
    int pml;
    int64_t psi_comp;
    const double* pml_bh;
    const double* pml_ch;
    const double* pml_be;
    const double* pml_ce;
    // fused 3D step only: material ids packed per cell, x = Ex | Ey << 8 |
    // Ez << 16 | Hx << 24, y = Hy | Hz << 8
    const uint2* idp;
    // fused 3D steps: per band of a variant, the planes [x, y) outside which
    // the band's region holds no field that can become nonzero (every E
    // component there and on the next plane is held at 0 by a perfect
    // conductor, so H keeps its initial 0 too); variant v's table starts at
    // zr_tab + zr_off[v].  zr_tab == nullptr: every plane is marched.
    const int2* zr_tab;
    int zr_off[8];
};
// Shape of fused 3D variant v: waves W, rows per wave B, steps per launch.
void f3d_shape(int variant, int* w, int* b, int* steps);



// 2D launchers.  `slots` lists the channel descriptors to advance (one
// thread-block row per slot).  pol is CF_POL_TM or CF_POL_TE.  mode 0 =
// regular step half, mode 1 = consistent start (H half for E-kind
// channels, E half for H-kind channels).
template <typename T>
hipError_t launch_h2d(int pol, int mode, T* fields, const ChanDev* ch, const int* slots, int nslots,
                      const Grid2D& g, const T* lut, hipStream_t s);
template <typename T>
hipError_t launch_e2d(int pol, int mode, T* fields, const ChanDev* ch, const int* slots, int nslots,
                      const Grid2D& g, const T* lut, hipStream_t s);

// Cylindrical (r, z) half steps of azimuthal order m for the listed
// channels (6-component blocks on a Grid2D with x = z, y = r); mode as for
// the 2D launchers.
// Reduced two-dimensional problems (cylindrical orders, k_z runs): coupling
// = m or k dx of the run, axis = 1 when row 0 is the symmetry axis, rows =
// 6 factors per row j in the field precision (see kernels_reduced.hip).
// cplx: complex (Bloch-periodic x) run, 12 values per cell (real part, then
// imaginary part), with the phase ph_c + i ph_s across the periodic x edge.
template <typename T>
hipError_t launch_hred(int mode, double coupling, int axis, T* fields, const ChanDev* ch, const int* slots,
                       int nslots, const Grid2D& g, const T* lut, const T* rows, double ph_c, double ph_s, int cplx,
                       hipStream_t s);
template <typename T>
hipError_t launch_ered(int mode, double coupling, int axis, T* fields, const ChanDev* ch, const int* slots,
                       int nslots, const Grid2D& g, const T* lut, const T* rows, double ph_c, double ph_s, int cplx,
                       hipStream_t s);

// Per-order tables of a reduced solve (cylindrical orders m, or k_z points):
// coefficient table of order q at lut + q * lut_stride (field precision),
// K(t_k) at ktab + q * ktab_stride, T_q steps of dt_q.
constexpr int kMaxOrders = 33;
struct RedOrders {
    const void* lut;
    int64_t lut_stride;
    const double* ktab;
    int64_t ktab_stride;
    int steps[kMaxOrders];
    double dt[kMaxOrders];
    // the six material ids of each cell in 4 bits each (component c at bit
    // 4 c; 15 stands for the wall id), or null when an id does not fit
    const uint32_t* idw;
    const void* rows;                 // 6 row factors per row (field precision)
    double coup[kMaxOrders];       // coupling of each order: m, or k dx
    double ph_c[kMaxOrders];       // Bloch phase across the periodic x edge (complex runs)
    double ph_s[kMaxOrders];
    int axis;                         // row 0 is the symmetry axis (cylindrical)
    int cplx;                         // complex fields (Bloch-periodic x)
};

// Resident cylindrical solve: one block per listed channel clears its
// field block, deposits the kick, takes the consistent start and all T_m
// steps of its order (ChanDev.order), projecting onto S and accumulating
// after each; acc/gamma as for launch_surface.  variant 1: fields in
// registers with an LDS exchange (used when the grid fits, else variant 2),
// 2: fields in global memory (L2-resident); 0 picks 1 when it fits.  *used
// receives the variant launched.
template <typename T>
hipError_t launch_red_resident(int variant, T* fields, const ChanDev* ch, const int* slots, int nslots,
                               const Grid2D& g, const RedOrders& ord, const SurfTables& t, double dA, double* acc,
                               double* gamma, int gamma_stride, hipStream_t s, int* used);

template <typename T>
hipError_t launch_kick(T* fields, const ChanDev* ch, const int* slots, int nslots, int max_uniq,
                       const SurfTables& t, hipStream_t s);

// Surface projection + g-weighted accumulation for step m (0-based sample
// index into ktab).  acc holds (sum, compensation) per channel descriptor.
// gamma, when non-null, receives Gamma at gamma[m * gamma_stride + slot].
template <typename T>
hipError_t launch_surface(const T* fields, const ChanDev* ch, const int* slots, int nslots,
                          const SurfTables& t, const double* ktab, int m, double dt, double dA,
                          double* acc, double* gamma, int gamma_stride, hipStream_t s);

template <typename T>
hipError_t launch_h3d(int mode, T* fields, T* psi, const ChanDev* ch, const int* slots, int nslots,
                      const Grid3D& g, const T* lut, hipStream_t s);
template <typename T>
hipError_t launch_e3d(int mode, T* fields, T* psi, const ChanDev* ch, const int* slots, int nslots,
                      const Grid3D& g, const T* lut, hipStream_t s);

// Fused launch over a work list of nwork items, all of polarization pol:
// every item advances its channel by min(kmax, remaining steps of its
// instance) steps starting at launch-clock step m, between its instance's
// two field buffers in the direction given by parity.
// Box of grid cells that holds every surface stencil point of a 3D solve:
// x0 .. x0 + bnx - 1 (likewise y, z), vol = bnx bny bnz.  A two-step fused
// 3D launch stores there the measured component of every channel after the
// first of its two steps: the channel whose field block is b (field_off =
// 6 ncell b) at shadow + b vol, cell (x, y, z) at
// ((z - z0) bny + (y - y0)) bnx + (x - x0).
struct ShadowBox {
    int x0, y0, z0, bnx, bny, bnz;
    int64_t vol;
};

// Fused 3D step (z-streaming; reads src, writes dst, CPML psi likewise).
// Usable for nx <= 256, z walls PEC or CPML.  f3d_steps(variant) time steps
// per launch: 1, or 2 for the two-step variants, which also fill `shadow`
// (see ShadowBox); a single-step launch ignores shadow.  f3d_single(v) is
// the single-step variant of the same band shape.
int f3d_variants();
int f3d_steps(int variant);
int f3d_single(int variant);
template <typename T>
bool f3d_usable(int variant, const Grid3D& g);
template <typename T>
hipError_t launch_f3d(int variant, const ChanDev* ch, const int* slots, int nslots, const Grid3D& g, const T* lut,
                      const T* src, T* dst, const T* psrc, T* pdst, T* shadow, const ShadowBox& sb,
                      hipStream_t s);
// Surface projection and accumulation of step m (as launch_surface) reading
// the measured component from the shadow box of a two-step launch.
template <typename T>
hipError_t launch_surface_box(const T* shadow, const ShadowBox& sb, const Grid3D& g, const ChanDev* ch,
                              const int* slots, int nslots, const SurfTables& t, const double* ktab, int m,
                              double dt, double dA, double* acc, double* gamma, int gamma_stride, hipStream_t s);

template <typename T>
hipError_t launch_tb2d(int variant, int pol, const ChanDev* ch, const WorkItem* work, int nwork,
                       const InstDev* inst, int kmax, int m, int parity, hipStream_t s);

}  // namespace cf
