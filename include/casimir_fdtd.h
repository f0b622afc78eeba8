/*
 * casimir_fdtd.h - C ABI of the MI355X (gfx950) time-domain Casimir-force
 * library.
 *
 * The library computes the Casimir force on an object by the time-domain
 * stress-tensor method of McCauley, Rodriguez, Joannopoulos and Johnson,
 * "Casimir forces in the time domain: Applications":
 *
 *   - one Yee-grid FDTD run per harmonic current source on the stress
 *     surface S (Sec. II, the harmonic expansion of the surface delta
 *     function; Sec. III A, the per-face cosine basis f_n),
 *   - with a uniform artificial conductivity sigma that makes the response
 *     decay (Sec. II),
 *   - recording the stress-tensor field correlations Gamma on S at every
 *     step and integrating them in time against the kernel g(-t)
 *     (Sec. II, eq. time-force; Appendix A, the closed forms of g).
 *
 * Conventions shared by every entry point:
 *   - Every function returns cf_status (CF_OK == 0) and never throws or
 *     aborts: bad input gives its status, a failed host allocation inside
 *     the library CF_E_BUDGET; cf_last_error() returns a thread-local
 *     message describing the most recent failure on the calling thread.
 *   - Units: hbar = c = eps_0 = mu_0 = 1.  Lengths are in units of the
 *     geometry (1/res per cell); time step dt = courant / res.
 *   - Arrays passed in are host memory, read during the call and copied;
 *     the caller keeps ownership.  Output arrays are host memory allocated
 *     by the caller, with their lengths passed; a length shorter than
 *     required gives CF_E_ARG and writes nothing.
 *   - Device memory: a solve needs cf_workspace_size() bytes of device
 *     memory.  The caller may pass its own allocation (e.g. a PyTorch tensor)
 *     as `workspace`; with workspace == NULL the library allocates and frees
 *     it itself.  Work is issued on opts->stream (a hipStream_t; NULL = the
 *     default stream) and the call returns after the results are on the
 *     host.
 *   - Results are deterministic: identical inputs and options give
 *     bitwise-identical outputs.
 */
#ifndef CASIMIR_FDTD_H
#define CASIMIR_FDTD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    CF_OK = 0,
    CF_E_ARG = 1,         /* invalid argument, shape or length                  */
    CF_E_CFL = 2,         /* courant number above the Yee stability limit       */
    CF_E_SURFACE = 3,     /* S leaves the grid or does not lie in one uniform medium */
    CF_E_BUDGET = 4,      /* workspace smaller than required / budget exceeded  */
    CF_E_NONFINITE = 5,   /* a force accumulator became NaN or infinite          */
    CF_E_DEVICE = 6,      /* HIP runtime error                                   */
    CF_E_CANCELLED = 7,   /* request cancelled before completion                 */
    CF_E_UNSUPPORTED = 8  /* option combination not implemented                  */
} cf_status;

/* Boundary per axis (both ends of the axis).  CF_BC_PML: a CPML
 * (Roden-Gedney, polynomial order 3, R0 = 1e-8, kappa = 1, alpha = 0) of
 * pml_cells cells inside the grid at both ends, backed by a PEC wall
 * (Sec. III B: open space around the bodies; Sec. III C: open tube ends).
 * 3D grids take it along z; Cartesian 2D and k_z problems along x and/or
 * y; cylindrical problems along the tube axis (x) only, the tube wall
 * staying PEC (CF_E_ARG at creation otherwise).  In 2D, k_z and
 * cylindrical problems the split half-step kernels carry the layers (the
 * fused and resident kernels do not); each cylindrical order uses the
 * profile of its own time step.  The kick and the consistent start stretch
 * their differences inside a layer as every later step does. */
enum { CF_BC_PEC = 0, CF_BC_PERIODIC = 1, CF_BC_PML = 2 };
/* Polarizations: 2D runs take CF_POL_TM, CF_POL_TE or both OR-ed; 3D runs CF_POL_3D. */
enum { CF_POL_TM = 1, CF_POL_TE = 2, CF_POL_3D = 4 };
/* Time kernel (Appendix A): general, or the 2D cross-section of a z-invariant
 * perfect-conductor system (Appendix A.2). */
enum { CF_KERNEL_GENERAL = 0, CF_KERNEL_ZINV2D = 1 };
/* Field precision.  The surface projection and the g-weighted time
 * accumulation are always FP64 (compensated). */
enum { CF_FP64 = 0, CF_FP32 = 1 };
/* Execution path: all channels advanced together (batched), or one channel
 * at a time with three kernel launches per time step (plain). */
enum { CF_PATH_BATCHED = 0, CF_PATH_PLAIN = 1 };

/* Component order of every per-component array: Ex, Ey, Ez, Hx, Hy, Hz. */
enum { CF_EX = 0, CF_EY, CF_EZ, CF_HX, CF_HY, CF_HZ };

/*
 * Coordinates (cf_grid.coord).  CF_COORD_CYLINDRICAL describes a problem
 * with cylindrical symmetry (Sec. III C; Appendix, harmonic expansion in
 * cylindrical coordinates): fields proportional to exp(i m phi) reduce to
 * the (r, z) half plane, solved once per azimuthal order m = 0..m_max.
 *   - ndim = 2; axis 0 is z (the symmetry axis, n[0] cells), axis 1 is r
 *     (n[1] cells); n[2] = 1.  bc[0] is CF_BC_PEC or CF_BC_PERIODIC; bc[1]
 *     must be CF_BC_PEC: a perfectly conducting tube wall at
 *     r = (n[1] - 1/2) / res.
 *   - The six component slots hold Ex = E_z, Ey = E_r, Ez = -i E_phi,
 *     Hx = -i H_z, Hy = -i H_r, Hz = H_phi (the phase factors make the
 *     reduced system real).  Components with doubled Yee offset 1 along
 *     axis 1 (Ey, Hx, Hz) sit at r = j / res, the others (Ex, Ez, Hy) at
 *     r = (j - 1/2) / res; row j = 0 of the latter lies outside the domain
 *     and stays zero.  comp_id uses the Cartesian index (j * n[0] + i).
 *   - The symmetry axis: H_z on it follows the circulation of E_phi around
 *     the disk of radius half a cell (m = 0) and is zero otherwise; E_r and
 *     H_phi on it are the next row's values for m = 1 and zero otherwise
 *     (the interpolation onto S applies this; the arrays hold zero there).
 */
enum { CF_COORD_CARTESIAN = 0, CF_COORD_CYLINDRICAL = 1, CF_COORD_KZ = 2 };

/*
 * CF_COORD_KZ describes a z-invariant two-dimensional problem solved at
 * Bloch wavevectors k_z along the invariant axis (Sec. III B: dielectrics
 * hybridize the polarizations, so every k_z is its own two-dimensional
 * simulation; Sec. III D: the force as an integral over the wavevectors).
 *   - ndim = 2, bc[0], bc[1] CF_BC_PEC or CF_BC_PERIODIC; the grid, the
 *     materials and S as for a Cartesian 2D problem.
 *   - Fields proportional to exp(i k z) with E_z, H_x, H_y carried as
 *     -i times their value: a real system in all six components, the k
 *     terms coupling E_x with H_y and E_y with H_x (at k = 0 it splits into
 *     TM and TE).
 *   - cf_surface.kz[q], kz_weight[q] (q < n_kz <= 33): the force is
 *     F = sum_q kz_weight[q] F(k_q), F(k) = (1/pi) sum_c s_c acc_c the
 *     two-dimensional force of the run at k (use the general kernel).  For
 *     the force per unit length, (1/pi) int_0^inf F(k) dk, the weights of a
 *     quadrature on [0, inf) times 1/pi.
 *   - Every k runs with the same time step and step count; courant must
 *     satisfy courant * v_max * sqrt(8 + (k_max / res)^2) / 2 < 1.
 *   - Channels, labels (q * n_harm + n) and signs (times kz_weight[q]) are
 *     ordered as for cylindrical orders.
 *   - Bloch-periodic x (Sec. III D, a cell periodic in x with period
 *     L = n[0] / res): kx[q] != 0 at any point makes the fields complex
 *     (quasi-periodic: F(x + L) = exp(i kx L) F(x)); bc[0] must be
 *     CF_BC_PERIODIC and S must not reach across the periodic x edge (no
 *     interpolation point beyond it), else CF_E_SURFACE.  Sources are real
 *     and the force takes the real part of the response (the -kx point is
 *     the complex conjugate: weight the pair accordingly).  Complex runs use
 *     12 values per cell and the global-memory resident kernel (or the
 *     split kernels).
 */

typedef struct cf_grid {
    int ndim;          /* 2 or 3                                                   */
    int n[3];          /* cells nx, ny, nz (nz == 1 when ndim == 2)               */
    double res;        /* cells per unit length                                    */
    int bc[3];         /* CF_BC_* per axis; 2D problems ignore bc[2]               */
    int pml_cells[3];  /* PML thickness in cells at each end of a CF_BC_PML axis   */
    int coord;         /* CF_COORD_* (0 = Cartesian)                               */
} cf_grid;

/*
 * Materials (Sec. III A uses PEC (eps = -inf) and PMC (mu = -inf) walls;
 * Sec. III E uses dielectrics).  comp_id[c] is a host array of
 * n[2]*n[1]*n[0] bytes (index (k*ny + j)*nx + i) giving the material of Yee
 * component c at cell (i, j, k); component c of a cell sits at the standard
 * Yee position (E_a half a cell along a, H_a half a cell along both other
 * axes).  NULL means id 0 everywhere.  eps[id] == -INFINITY marks a perfect
 * electric conductor (E held at 0), mu[id] == -INFINITY a perfect magnetic
 * conductor (H held at 0).  n_materials <= 254.
 */
typedef struct cf_materials {
    int n_materials;
    const double* eps;
    const double* mu;
    const uint8_t* comp_id[6];
    /* Dispersive materials (Sec. III B: a fitted Lorentz model, continued onto
     * the complex conductivity contour).  Material id has the permittivity
     *   eps(omega) = eps[id] + sum_j d_eps_j w0_j^2 / (w0_j^2 - omega^2),
     * d_eps_j = lorentz_deps[id * n_lorentz + j], w0_j = lorentz_w0[...]
     * (w0 in radians per unit time, c = 1; a term with d_eps = 0 is absent).
     * On the contour omega^2 = xi^2 + i sigma xi every term becomes a
     * polarization P with P'' + sigma P' + w0^2 P = d_eps w0^2 E, and
     * D = eps[id] E + sum P carries the conductivity of E-current runs.
     * n_lorentz = 0 (or NULL arrays): no dispersion.  Limits: Cartesian 2D
     * and k_z problems only (3D and cylindrical: CF_E_UNSUPPORTED at
     * validation); S must lie in a non-dispersive medium (CF_E_SURFACE); at
     * most 4 terms per material.  Stability (CF_E_CFL otherwise): w0 dt < 2
     * for every term, and the fastest grid mode of the coupled field and
     * polarizations stays below 2 / dt:
     *   eps X - K^2 / mu + sum_j d_eps_j w0_j^2 X / (w0_j^2 - X) > 0,
     * X = 4 / dt^2, K^2 = (8 + (k_max dx)^2) / dx^2 in 2D (k_max: the largest
     * |k_z| of a k_z problem), for each dispersive material (eps, mu); a
     * strong term lowers the stable Courant number well below the Yee limit
     * at eps.  Dispersive problems run on the split half-step kernels (the
     * fused and resident kernels do not take them) and are not served
     * (CF_E_UNSUPPORTED). */
    int n_lorentz;
    const double* lorentz_deps;
    const double* lorentz_w0;
} cf_materials;

/*
 * Stress surface S (Sec. III: a rectangle / box with a cosine basis on each
 * face).  lo/hi are integer cell coordinates of the box corners.  Each face
 * is sampled at cell midpoints along its tangential axes; an axis spanned
 * completely while periodic has no faces.  n_harm cosine harmonics are used
 * per tangential axis (clamped per face to its sample count: the discrete
 * cosine basis has no more orthonormal members).  S must lie at least one
 * cell inside one uniform, non-conducting medium, else CF_E_SURFACE.
 */
typedef struct cf_surface {
    int lo[3];
    int hi[3];
    int n_harm;
    int force_axis;    /* 0, 1 or 2 */
    int m_max;         /* cylindrical problems: azimuthal orders 0..m_max (<= 32) */
    const double* kz;        /* CF_COORD_KZ problems: the wavevectors k_q (host, copied) */
    const double* kz_weight; /* and their weights                                        */
    int n_kz;                /* number of wavevectors (1..33)                            */
    const double* kx;        /* CF_COORD_KZ: Bloch wavevector along x per point, or NULL  */
} cf_surface;

/*
 * Cylindrical problems.  S is the surface of revolution of the (z, r)
 * rectangle lo..hi: lo[1] = 0 closes it on the axis (no inner face),
 * hi[1] = n[1] extends it to the tube wall (no outer face; the stress on a
 * conducting wall has no axial component).  Samples along r sit at
 * r = k + 1/2 cells; a face ending at the wall ends with a half-cell sample
 * at r = n[1] - 1 of weight 1/2.  The per-face basis is the cosine basis
 * made orthonormal under these quadrature weights (Gram-Schmidt); the line
 * element is the Cartesian ds of the (r, z) plane (the Jacobian r cancels).
 * force_axis must be 0 (the axial force).  Each order m runs on its own time
 * step: courant_m = courant for m <= 1 and min(courant, 1/(1 + m)) above
 * (the m/r couplings raise the scheme's largest frequency), for
 * T_m = round(n_steps courant / courant_m) steps (the same physical time),
 * with K sampled at its own steps.  The force is
 *   F = (1/pi) sum_m w_m sum_c s_c sum_k dt_m K(t_k) Gamma_c(t_k),
 * w_0 = 1, w_m>0 = 2 (the -m term is the conjugate of the +m term).
 * Options (cylindrical and k_z problems alike): pol = CF_POL_3D (all six
 * components); cylindrical runs need courant <= 0.5.  The convergence stop
 * counts steps on the axis of n_steps: after d of them every order has run
 * floor(d T_m / n_steps) of its own steps (the same physical time, to one
 * step of each order), and F(T') sums the channels there; it applies to the
 * resident kernels with one wave of channels.  The server runs these
 * problems as one whole solve per request.  Execution: by
 * default one launch per wave of resident channels (any mix of orders),
 * each block carrying one channel through all its steps; tile_variant 1
 * keeps the fields in registers with an LDS exchange (real runs: grids of up
 * to 10240 cells in FP32, 6144 in FP64; complex runs, both parts in
 * registers: 6144 and 3072; and only when the device's LDS holds the
 * exchange array of 3 values per cell and part; otherwise variant 2 runs),
 * 2 keeps them in global memory, 0 picks 1 when it fits.  CF_FLAG_SPLIT (and CF_PATH_PLAIN) use one launch per half
 * step.  All give bitwise-identical results; cf_result.fused/tile_variant
 * report the variant that ran.
 */

/* CF_FLAG_KEEP_GAMMA keeps Gamma_c(t_m) for the gamma/trace outputs.
 * CF_FLAG_TIME_STENCIL brackets sampled launches of the field-update
 * kernel with HIP events on the solve's stream and reports their average
 * duration (cf_result.stencil_ms_avg); the stepping loop is otherwise
 * unchanged.
 * CF_FLAG_SPLIT makes the batched path use one launch per half step instead
 * of the fused multi-step kernel (same arithmetic, bitwise-equal results).
 * CF_FLAG_GRAPH captures the fused stepping loop of each channel wave (and
 * of a batched solve) into a HIP graph and launches it as one graph instead
 * of one kernel launch per K steps (same kernels and arguments, bitwise-equal
 * results; ignored together with CF_FLAG_TIME_STENCIL).
 * CF_FLAG_INJECT_NAN is a fault-injection hook for failure-handling tests:
 * the kick of the first channel run is scaled by NaN, so its accumulator
 * becomes non-finite and the solve (or served request) fails with
 * CF_E_NONFINITE; nothing else changes. */
enum { CF_FLAG_KEEP_GAMMA = 1, CF_FLAG_TIME_STENCIL = 2, CF_FLAG_SPLIT = 4, CF_FLAG_INJECT_NAN = 8,
       CF_FLAG_GRAPH = 16 };

typedef struct cf_opts {
    double sigma;       /* uniform conductivity (decay rate), >= 0            */
    double courant;     /* dt * res; must be below 1/sqrt(ndim) / max speed   */
    int n_steps;        /* time steps T (samples at t_m = m dt, m = 1..T)     */
    int pol;            /* CF_POL_* (bitmask for 2D)                          */
    int kernel;         /* CF_KERNEL_*                                        */
    int precision;      /* CF_FP64 or CF_FP32                                 */
    int path;           /* CF_PATH_*                                          */
    int flags;          /* CF_FLAG_*                                          */
    const int* channel_subset;  /* optional: run only these channel indices  */
    int n_subset;               /* length of channel_subset (0 = all)         */
    void* stream;       /* hipStream_t, or NULL for the default stream        */
    int max_resident;   /* channels whose fields are on the device at once;   */
                        /* the channels run in consecutive waves of this many */
                        /* (0 = all at once).  Bounds the workspace of large  */
                        /* 3D problems; results do not depend on it.          */
    int tile_variant;   /* fused kernel variant (2D tile shape, or 3D band shape): 0 = autotune (timed on */
                        /* the solve's own data, cached per shape in the      */
                        /* process and in $CF_AUTOTUNE_CACHE when set),       */
                        /* k >= 1 = variant k-1.  3D: 1..4 one time step per  */
                        /* launch, 5..6 two (paired steps; an odd last step   */
                        /* on the one-step shape).  Results do not depend on it. */
    double stop_tol;    /* time-convergence stop (Appendix A, Fig. 12): 0 = off.  Every */
    int stop_every;     /* stop_every steps (0: 500) the partial force F(T') is formed   */
                        /* from the FP64 accumulators; the run ends once two consecutive */
                        /* windows change it by at most stop_tol |F(T')|.  Used when all */
                        /* channels are resident at once (one wave); turns off           */
                        /* CF_FLAG_GRAPH.  cf_result.n_steps_run gives the steps run.    */
} cf_opts;

typedef struct cf_info {
    int n_channels;        /* channels of the full problem                     */
    int n_faces;
    int per_harmonic_len;  /* entries of cf_result.per_harmonic                */
    int n_comp;            /* field components per channel (3 in 2D, 6 in 3D) */
    size_t workspace_bytes;
    double eps_s, mu_s;    /* medium S lies in                                 */
    int n_steps_max;       /* time steps of the longest run (n_steps unless    */
                           /* a cylindrical order runs on a smaller step)      */
} cf_info;

/*
 * Outputs.  force is F along force_axis (per unit z-length for 2D runs).
 * per_harmonic[k] is the contribution of harmonic label k (n in 2D,
 * m*n_harm + n in 3D; Fig. 5), per_face[f] of face f = 2*axis + (side > 0),
 * per_channel[c] = sum_m dt K(t_m) Gamma_c(t_m) (unsigned, without 1/pi),
 * gamma[m*C + c] = Gamma_c(t_{m+1}) (needs CF_FLAG_KEEP_GAMMA) and
 * trace[m] = F after m+1 steps (Fig. 12; needs CF_FLAG_KEEP_GAMMA).
 * Optional arrays may be NULL.  With a channel subset, per_channel and gamma
 * follow the subset order and force/per_* sum over the subset only.
 * Cylindrical problems: gamma has cf_info.n_steps_max rows, row k holding
 * step k + 1 of each channel's own order (zero past its T_m); trace is not
 * defined (orders advance on different time steps) and is left untouched.
 */
typedef struct cf_result {
    double force;
    double* per_harmonic; int per_harmonic_len;
    double* per_face;     int per_face_len;
    double* per_channel;  int per_channel_len;
    double* gamma;        long long gamma_len;
    double* trace;        int trace_len;
    int n_channels_run;
    double cell_updates;  /* channels * cells * steps advanced               */
    double device_ms;     /* time of the stepping loop on the stream         */
    double stencil_ms_avg;       /* mean duration of one field-update launch (CF_FLAG_TIME_STENCIL) */
    int stencil_samples;         /* launches timed                                                  */
    int stencil_launches;        /* field-update launches in the solve                              */
    double stencil_alg_bytes;    /* algorithmic HBM bytes of one field-update launch:               */
                                 /* one read + one write of the state it advances                   */
    double stencil_cell_updates; /* cell-updates one field-update launch performs                   */
    int fused;                   /* 1 when the fused multi-step kernel advanced the fields          */
    int tile_variant;            /* fused kernel variant used (1-based), 0 if not fused             */
    int tile_halo;               /* steps per fused launch of that variant                          */
    int n_steps_run;             /* time steps run (< n_steps when the convergence stop ended it)   */
    double advanced_cell_updates; /* cell-updates the field kernels actually performed: below        */
                                  /* cell_updates when the fused 2D kernel skips rows that hold only  */
                                  /* perfect conductor (fields identically 0 there)                   */
} cf_result;

typedef struct cf_problem cf_problem;

/* Build a problem: copies the inputs, rasterizes walls, builds S, the
 * per-face cosine basis and the interpolation tables.  *out receives a
 * handle to free with cf_problem_destroy.  CF_E_ARG on bad shapes/ids,
 * CF_E_SURFACE when S is invalid. */
cf_status cf_problem_create(const cf_grid* grid, const cf_materials* mats,
                            const cf_surface* surf, cf_problem** out);
cf_status cf_problem_destroy(cf_problem* p);

/* Sizes and medium for a solve with these options (no device work). */
cf_status cf_problem_info(const cf_problem* p, const cf_opts* opts, cf_info* out);

/* Channel table (Sec. II, the stress-tensor components as separate runs):
 * for channel c, face index, harmonic label, kind (0 = E-current source,
 * 1 = H-current source), source and measured component (CF_EX..CF_HZ) and
 * sign (outward-normal side times stress coefficient).  Arrays of length
 * >= n (n = cf_info.n_channels); NULL arrays are skipped.  Cylindrical
 * problems list the channels of order 0, then 1, ... m_max; their label is
 * m * n_harm + n and their sign includes the order weight w_m. */
cf_status cf_channel_table(const cf_problem* p, const cf_opts* opts, int n, int* face,
                           int* label, int* kind, int* src, int* meas, double* sign);

/* Validation: CFL limit, surface placement, option ranges (no device work). */
cf_status cf_validate(const cf_problem* p, const cf_opts* opts);

/* Device bytes a solve with these options needs. */
cf_status cf_workspace_size(const cf_problem* p, const cf_opts* opts, size_t* bytes);

/* Blocking force solve (Sec. II algorithm) on opts->stream.  workspace is a
 * device pointer of ws_bytes >= cf_workspace_size() bytes, or NULL. */
cf_status cf_solve(cf_problem* p, const cf_opts* opts, void* workspace, size_t ws_bytes,
                   cf_result* out);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): cf_solve
 * with the workspace taken from a fixed array of CF_STATIC_WORKSPACE_BYTES
 * (64 MiB) in device memory that the library holds on each device it runs
 * on until the process ends.  It calls no hipMalloc or hipFree.  A solve
 * whose cf_workspace_size() exceeds the array gives CF_E_BUDGET (use
 * cf_solve); CF_FLAG_GRAPH gives CF_E_UNSUPPORTED (instantiating a graph
 * allocates).  Results are bitwise those of cf_solve with the same options.
 * Every call on a device shares that device's array, which keeps the last
 * call's contents (each call clears what it reads before writing it): calls
 * on one device are serialized by a lock inside the library, and work that
 * another process or module queues on the same memory is not possible, but a
 * caller must not read the array's previous contents as a result. */
#define CF_STATIC_WORKSPACE_BYTES ((size_t)64 << 20)
cf_status cf_solve_static(cf_problem* p, const cf_opts* opts, cf_result* out);

/* Batched solve: n problems (for instance a sweep of sidewall separations)
 * with the same options, advanced together.  2D problems whose stress
 * surfaces fit the fused kernel's tiles share one fused launch sequence:
 * every launch advances the channels of all of them (each problem keeps its
 * own grid, materials, surface and coefficient table).  Reduced problems
 * (cylindrical, k_z, Bloch), when there are two or more, are solved
 * concurrently: up to four host threads, each with a stream of its own
 * (default priority) that first waits for the work queued on opts->stream,
 * take them in turn, each result bitwise as by cf_solve.  Any other problem
 * is solved on its own as by cf_solve.  outs[i] receives problem i's result;
 * channel_subset, max_resident and CF_FLAG_KEEP_GAMMA are not used.
 * workspace is NULL (allocated internally) or a device buffer of at least
 * cf_batch_workspace_size() bytes. */
cf_status cf_batch_workspace_size(cf_problem* const* probs, int n, const cf_opts* opts, size_t* bytes);
cf_status cf_batch_solve(cf_problem* const* probs, int n, const cf_opts* opts, void* workspace,
                         size_t ws_bytes, cf_result* outs);

/* The time kernel K(t_m) = 2 pi Im g(-t_m), t_m = m dt for m = 1..n
 * (Appendix A, general and z-invariant forms), written to out[m-1]. Host
 * only. */
cf_status cf_kernel_table(int kernel, double sigma, double dt, int n, double* out);

/* Message describing the last failure on this thread ("" if none). */
const char* cf_last_error(void);

/* ---- Serving: continuous batching of force solves (one GPU) ------------
 *
 * A server owns a device memory budget and a scheduler thread.  Requests
 * (one problem + options each, the whole Sec. II force computation) are
 * queued in arrival order; a request enters as soon as its memory fits the
 * budget (a later request may pass an earlier one that does not fit yet) and
 * leaves when all its time steps have run, returning its memory.  In every
 * scheduler tick the 2D requests whose stress surface fits a fused tile
 * share fused launches and advance steps_per_tick steps; every other
 * resident request (3D, wider 2D) advances the steps that an equal share of
 * the tick's device time buys it, from its measured time per step.
 * Cylindrical and k_z requests (Sec. III B, III C: one launch runs every
 * step of a channel) run their whole solve as cf_solve in one tick, on
 * their region of the budget; the convergence stop is not available for
 * them.  Problems with dispersive materials, and Cartesian 2D problems
 * with in-plane PML layers, are not served (CF_E_UNSUPPORTED).
 * A request's arithmetic does not depend on what else is resident: a result
 * is bitwise the same alone and in any mix, and equals cf_solve with the
 * same options and tile_variant (fused 2D and 3D) or CF_FLAG_SPLIT (wider
 * 2D).
 *
 * Ownership: cf_server_submit copies the problem into the request, so the
 * caller may destroy its handle as soon as the call returns.  A request that
 * has finished keeps only what its result needs.  cf_server_destroy cancels
 * what is still queued or running and must not overlap other calls on the
 * same server.  All other calls are thread-safe. */
typedef struct cf_server cf_server;

enum {
    CF_REQ_QUEUED = 0,
    CF_REQ_RUNNING = 1,
    CF_REQ_DONE = 2,
    CF_REQ_FAILED = 3,
    CF_REQ_CANCELLED = 4
};

typedef struct cf_server_info {
    uint64_t submitted, completed, failed, cancelled;
    int queued, running;       /* requests waiting / resident now */
    size_t bytes_in_use;       /* of the request arena */
    size_t budget;             /* request arena size (budget minus server tables) */
    int64_t clock_steps;       /* time steps the scheduler clock has advanced */
    double busy_s;             /* wall time spent in ticks */
    int steps_per_tick;
} cf_server_info;

/* Create a server.  hbm_budget_bytes: device memory for the server's tables
 * and every resident request; arena: a device buffer of that size, or NULL
 * to allocate one.  precision: CF_FP32 / CF_FP64 for every request.
 * tile_variant: fused kernel variant (1-based, as in cf_opts) used for all
 * fused requests, 0 for the default.  stream: hipStream_t, or NULL for a
 * stream of the server's own.  CF_E_BUDGET when the budget cannot hold the
 * server's tables. */
cf_status cf_server_create(size_t hbm_budget_bytes, int precision, int tile_variant, void* arena,
                           void* stream, cf_server** out);

/* Queue a request; *ticket identifies it.  opts->precision must match the
 * server's, path must be CF_PATH_BATCHED, channel_subset empty;
 * opts->max_resident bounds the channel waves of non-fused requests (0:
 * all channels, halved until the request fits the budget).  CF_E_BUDGET
 * when the request can never fit. */
cf_status cf_server_submit(cf_server* s, cf_problem* p, const cf_opts* opts, uint64_t* ticket);

/* State of a request (CF_REQ_*); when done, *out (may be NULL) receives its
 * result as from cf_solve (device_ms = wall time from admission to
 * completion, except for cylindrical and k_z requests, whose device_ms is
 * their cf_solve's).  gamma and trace are not kept (CF_E_ARG when asked);
 * short per_* arrays give CF_E_ARG.  Returns the request's error for failed
 * / cancelled ones. */
cf_status cf_server_poll(cf_server* s, uint64_t ticket, int* state, cf_result* out);

/* As cf_server_poll after waiting up to timeout_s seconds (< 0: no limit)
 * for the request to finish. */
cf_status cf_server_wait(cf_server* s, uint64_t ticket, double timeout_s, int* state, cf_result* out);

/* Ask for a request to stop: a queued one leaves at once, a running one at
 * the end of the current tick; its state becomes CF_REQ_CANCELLED. */
cf_status cf_server_cancel(cf_server* s, uint64_t ticket);

/* Submission, admission and completion times of a request (seconds on a
 * monotonic clock; 0 when not reached yet). */
cf_status cf_server_times(cf_server* s, uint64_t ticket, double* submit_s, double* admit_s,
                          double* done_s);

cf_status cf_server_stats(cf_server* s, cf_server_info* out);
cf_status cf_server_destroy(cf_server* s);

#ifdef __cplusplus
}
#endif

#endif /* CASIMIR_FDTD_H */
