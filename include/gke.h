/*
 * gke.h -- C ABI of the MI355X (gfx950) GKE two-point-statistics library.
 *
 * The library computes the terms of the Generalised Kolmogorov Equation for
 * plane channel flow (Gatti, Remigi, Chiarini, Cimarelli, Quadrio, "An
 * efficient numerical method for the Generalised Kolmogorov Equation"):
 * the scale energy <du^2> (eq. du2) and every flux and source component of
 * eqs. scale-flux, physical-flux and source, on the four-dimensional domain
 * (rx, rz, Y1, Y2) (Section "Structure of the GKE computer code": Y1 = Y - ry/2,
 * Y2 = Y + ry/2).  Correlations in the homogeneous directions x, z are
 * computed through the Parseval identity (Section "Products instead of
 * correlations"); derivatives along Y1, Y2 use an explicit five-point stencil
 * on the nonuniform y grid (Section "Step 3").
 *
 * Problem statement (Section "General structure of the program"): a database
 * of snapshots of (u~, v~, w~, p~) on a Cartesian grid, periodic in x and z,
 * nonuniform in y.  Step 1 scans it for the means, Step 2 scans it again and
 * averages the two-point statistics, Step 3 takes the wall-normal derivatives.
 * This ABI maps the two scans onto two sequences of gke_accumulate calls
 * separated by gke_begin_stats, and Step 3 onto gke_finalize.
 *
 * Conventions
 *   grid      x_m = m Lx/Nx, z_n = n Lz/Nz, nodes y[0..Ny) strictly increasing;
 *   fields    device arrays [Ny][Nz][Nx] row-major (x fastest), F64 or F32;
 *   average   <.> = mean over the Nx*Nz points of a plane (periodic
 *             wrap-around of separations) and over the snapshots;
 *   rho = 1   (the pressure flux is 2<dp dv>);
 *   separations are grid multiples rx = p Lx/Nx, rz = q Lz/Nz; an index
 *             q >= Nz/2 stands for the negative separation (q - Nz) Lz/Nz;
 *   x- and z-derivatives are spectral with a zero multiplier at the Nyquist
 *             wavenumber; y-derivatives use the five-point stencil (centred in
 *             the interior, shifted to the five nodes nearest a wall).
 *
 * Errors: every call returns a gke_status; no exception crosses the ABI.
 * gke_last_error(plan) describes the last failure on that plan.  A plan is
 * not thread-safe; separate plans are independent.  Work is enqueued on the
 * plan's HIP stream; only gke_begin_stats, gke_finalize, gke_get_profiles and
 * gke_destroy synchronise it.
 */
#ifndef GKE_H
#define GKE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct gke_plan_s *gke_plan_t;

typedef enum {
    GKE_OK = 0,
    GKE_ERR_ARG = 1,          /* invalid argument (shape, pointer, value) */
    GKE_ERR_STATE = 2,        /* call not allowed in the plan's current state */
    GKE_ERR_OOM = 3,          /* workspace missing or too small */
    GKE_ERR_HIP = 4,          /* a HIP runtime call or kernel launch failed */
    GKE_ERR_UNSUPPORTED = 5   /* valid request this build does not implement */
} gke_status;

/* option keys for gke_set_option (allowed before gke_set_workspace) */
enum {
    GKE_OPT_DTYPE = 1,        /* input storage: GKE_DTYPE_F64 (default) or GKE_DTYPE_F32 */
    GKE_OPT_PRECISION = 2,    /* rank-k arithmetic: GKE_PREC_FP64 (default) or GKE_PREC_BF16X3 */
    GKE_OPT_CHUNK = 3,        /* snapshots per cross-spectral batch, even, 2..4096 (default 64);
                                 0: the most whose spectra fit 96 GiB, in [8, 512] */
    GKE_OPT_PAIR_BATCH = 4,   /* plane pairs per finalize batch, 0 = all at once (default) */
    GKE_OPT_TIMING = 5,       /* 1: record HIP events around every kernel launch (any time) */
    GKE_OPT_MIRROR = 6,       /* 1: average every term with the reflected pair (below) */
    GKE_OPT_DOMAIN = 7,       /* output domain, GKE_DOMAIN_* (default ALLPAIRS_HALFRX) */
    GKE_OPT_SLAB = 8,         /* output Y1 rows per slab, 0 = all rows in one slab (default) */
    GKE_OPT_RESIDUAL = 9,     /* 1: reserve what gke_finalize needs to write the budget
                                 residual (gke_terms.residual; all-pairs mode only) */
    GKE_OPT_HOST_STAGING = 10,/* device staging buffers for host outputs (gke_terms.on_device
                                 = 0): 0 (default, device outputs only), 1, or 2 (the copies
                                 of one finalize overlap the next slab's scan) */
    GKE_OPT_STEP1 = 11,       /* 1: reserve the buffers of gke_reconstruct */
    /* block shapes for an autotuner (0: the built-in rule; gke_get_option
       reports the shape in effect once the workspace is sized): */
    GKE_OPT_TUNE_ZPLANES = 12,/* at most this many planes per z-transform block (1..64) */
    GKE_OPT_TUNE_KZPAIRS = 13,/* pairs per kz-finalize block (even, within its LDS) */
    GKE_OPT_TUNE_KXTRANS = 14 /* packed transforms per kx-finalize block (within its LDS) */
};
enum { GKE_DTYPE_F64 = 0, GKE_DTYPE_F32 = 1 };
enum { GKE_PREC_FP64 = 0, GKE_PREC_BF16X3 = 1 };

/* Mirror average (GKE_OPT_MIRROR = 1; Section "Step 2": one half of the
 * channel is used to double the sample, with the sign of each term set by its
 * symmetry under the inversion of y, Section "Exploiting symmetries"):
 *   Tbar(Y1, Y2; rx, rz) = (T(Y1, Y2) + sigma_y T(2h - Y1, 2h - Y2)) / 2,
 * sigma_y = -1 for T5, T6, T9, T10, T11 (an odd number of wall-normal
 * components) and +1 for the others.  Needs a y grid symmetric about its
 * centre to 1e-13 of its length; plane j reflects to Ny - 1 - j.
 *
 * Output domains (GKE_OPT_DOMAIN), for the pairs of one slab:
 *   GKE_DOMAIN_ALLPAIRS_HALFRX   Y1 in the slab, every Y2, rx >= 0 (Nx/2 + 1 columns);
 *   GKE_DOMAIN_Y1LEY2_FULLR      Y1 in the slab, Y2 >= Y1, every rx (Nx columns);
 *   GKE_DOMAIN_FUNDAMENTAL_FULLR Y1 <= h (index <= (Ny - 1)/2) in the slab,
 *                                Y1 <= Y2 <= 2h - Y1, every rx; needs MIRROR = 1
 *                                (Section "Exploiting symmetries": the terms
 *                                outside follow from the symmetries).
 * Slabs (GKE_OPT_SLAB = R > 0): the output rows of the domain are cut into
 * slabs of R rows (Section "Undersampling and parallelisation": the result
 * space split into wall-normal slices, independent thanks to the local
 * finite-difference stencil); each slab needs its own second scan, see
 * gke_begin_slab.  The accumulators then cover only the slab's rows, their
 * five-point neighbours and (mirror) the reflected rows. */
enum { GKE_DOMAIN_ALLPAIRS_HALFRX = 0, GKE_DOMAIN_Y1LEY2_FULLR = 1,
       GKE_DOMAIN_FUNDAMENTAL_FULLR = 2 };

/* term slots: the fourteen components of the budget, T1..T14 -> 0..13
 *   GKE_T_DU2      <du_i du_i>                    (eq. du2)
 *   GKE_T_PHIX_T   <du^2 du>                      (eq. scale-flux, turbulent, x)
 *   GKE_T_PHIX_M   <du^2 dU>                      (eq. scale-flux, mean flow)
 *   GKE_T_PHIX_V   -2 nu d<du^2>/drx              (eq. scale-flux, viscous, x)
 *   GKE_T_PHIY_T   <du^2 dv>                      (eq. scale-flux, turbulent, y)
 *   GKE_T_PHIY_V   -2 nu d<du^2>/dry              (eq. scale-flux, viscous, y)
 *   GKE_T_PHIZ_T   <du^2 dw>                      (eq. scale-flux, turbulent, z)
 *   GKE_T_PHIZ_V   -2 nu d<du^2>/drz              (eq. scale-flux, viscous, z)
 *   GKE_T_PHI_T    <v* du^2>                      (eq. physical-flux, turbulent)
 *   GKE_T_PHI_P    2 <dp dv>                      (eq. physical-flux, pressure)
 *   GKE_T_PHI_V    -(nu/2) d<du^2>/dY             (eq. physical-flux, viscous)
 *   GKE_T_XI_P1    -2 <du dv> (dU/dy)*            (eq. source, production 1)
 *   GKE_T_XI_P2    -2 <du v*> d(dU/dy)            (eq. source, production 2)
 *   GKE_T_XI_D     -4 <eps*>                      (eq. source, dissipation)
 * Totals: Phi_rx = T2+T3+T4, Phi_ry = T5+T6, Phi_rz = T7+T8,
 *         phi = T9+T10+T11, xi = T12+T13+T14. */
enum {
    GKE_T_DU2 = 0, GKE_T_PHIX_T, GKE_T_PHIX_M, GKE_T_PHIX_V, GKE_T_PHIY_T, GKE_T_PHIY_V,
    GKE_T_PHIZ_T, GKE_T_PHIZ_V, GKE_T_PHI_T, GKE_T_PHI_P, GKE_T_PHI_V, GKE_T_XI_P1,
    GKE_T_XI_P2, GKE_T_XI_D, GKE_NTERMS
};

/* Output of gke_finalize.  Each non-NULL t[i] is a caller-owned array of
 * dtype GKE_OUT_F64 (default) or GKE_OUT_F32 (every value is assembled in
 * FP64 and rounded once when stored; in the all-pairs mode T6 and T11 are
 * then formed from the rounded <du^2> and the residual from the rounded
 * maps), on the device (on_device = 1) or on the host (on_device = 0: needs
 * GKE_OPT_HOST_STAGING; the maps are written to a device staging buffer and
 * copied on a stream of the library's own, so that gke_finalize returns once
 * the maps are computed while the copies run; pinned host memory lets them
 * overlap the caller's next work; the host arrays are complete after
 * gke_wait_outputs, the next gke_finalize into the same staging buffer, or
 * gke_destroy).  Default (no mirror, all-pairs domain, one slab): maps T1..T13 are
 * laid out [Y1 0..Ny)[Y2 0..Ny)[q 0..Nz)[p 0..Nx/2] (all ordered pairs, the
 * half plane rx >= 0; the half rx <= 0 of pair (Y1,Y2) is the half rx >= 0 of
 * pair (Y2,Y1) by the r-inversion symmetry of Section "Exploiting
 * symmetries"), and T14, which does not depend on r, is laid out [Y1][Y2].
 * With mirror, another domain or slabs: the maps of the current slab are laid
 * out [n 0..npairs)[q 0..Nz)[p 0..width) with the slab's output pairs in the
 * order of gke_slab_pairs, width = Nx/2 + 1 (ALLPAIRS_HALFRX) or Nx (FULLR
 * domains), and T14 is laid out [n].  With rx / rz undersampling the q and p
 * extents are the kept rows and columns (gke_sample_indices).  on_device must be 1. */
enum { GKE_OUT_F64 = 0, GKE_OUT_F32 = 1 };
/* Budget residual (optional, gke_terms.residual; needs GKE_OPT_RESIDUAL = 1
 * and the all-pairs mode): the left-hand side minus the right-hand side of
 * the budget in conservative form (eq. GKE-conservative, the validation of
 * Section "GKE and turbulence physics"),
 *   Res = d(T2 + T3 + T4)/drx + d(T7 + T8)/drz + (d/dY2 - d/dY1)(T5 + T6)/2
 *         + (d/dY1 + d/dY2)(T9 + T10 + T11) - (T12 + T13 + T14),
 * with spectral rx, rz derivatives (zero multipliers at the Nyquist
 * wavenumbers) and the five-point stencil along Y1 and Y2, laid out like the
 * maps T1..T13.  It is assembled from the caller's maps, so T1, T5, T6, T9,
 * T10, T11, T12 and T13 must be requested too (else GKE_ERR_ARG). */
typedef struct {
    void *t[GKE_NTERMS];
    int on_device;      /* 1: device arrays; 0: host arrays */
    int dtype;          /* GKE_OUT_F64 (0) or GKE_OUT_F32 (1) */
    void *residual;     /* budget residual map, or NULL */
} gke_terms;

/* profile rows returned by gke_get_profiles, each of length Ny (FP64):
 * U V W P = means (Section "Step 1"), S = dU/dy (five-point stencil),
 * q = <u'_i u'_i>, uv = <u'v'>, pv = <p'v'>, Tx Ty Tz = <q u'_j>,
 * eps = nu <du'_i/dx_j du'_i/dx_j> (pseudo-dissipation, below eq. GKE). */
enum { GKE_P_U = 0, GKE_P_V, GKE_P_W, GKE_P_P, GKE_P_S, GKE_P_Q, GKE_P_UV, GKE_P_PV,
       GKE_P_TX, GKE_P_TY, GKE_P_TZ, GKE_P_EPS, GKE_NPROF };

/* Create a plan for an Nx x Ny x Nz grid.
 *   y   host array of Ny strictly increasing wall-normal nodes (copied);
 *   Nx, Nz even, >= 4, with no prime factor other than 2, 3, 5; Ny >= 5;
 *   Lx, Lz > 0 box lengths; nu > 0 kinematic viscosity.
 * On success *out receives the plan (release with gke_destroy).
 * Errors: GKE_ERR_ARG on any violation (then *out is NULL). */
gke_status gke_plan(int Nx, int Ny, int Nz, const double *y, double Lx, double Lz,
                    double nu, gke_plan_t *out);

/* Set an option (keys above) before gke_set_workspace.
 * Errors: GKE_ERR_ARG (unknown key, bad value), GKE_ERR_STATE (too late),
 * GKE_ERR_UNSUPPORTED (value not built). */
gke_status gke_set_option(gke_plan_t plan, int key, int64_t value);

/* Value of an option in effect: after gke_workspace_size or
 * gke_set_workspace, GKE_OPT_CHUNK reports the chunk chosen for 0.
 * Errors: GKE_ERR_ARG (NULL, unknown key). */
gke_status gke_get_option(gke_plan_t plan, int key, int64_t *value);

/* rx / rz undersampling (Section "Undersampling and parallelisation": the
 * correlations are always computed on the full grid and the stored maps keep
 * full resolution below a first threshold of the separation, one point in s1
 * between the two thresholds and one in s2 above the second; it drops output
 * points only, so every derivative -- the spectral rx, rz ones of T4, T8 and
 * of the residual, the five-point Y ones -- is taken at full resolution).
 * dir = 0: rx, dir = 1: rz.  In grid-index units, a separation of signed
 * index k (k = n, or n - N for n past N/2) is kept iff |k| < t1, or
 * t1 <= |k| < t2 and |k| is a multiple of s1, or |k| >= t2 and |k| is a
 * multiple of s2.  Default (t1, t2, s1, s2) = (0, 0, 1, 1): every separation.
 * The output maps then hold [..][nrz][nrx] over the kept rows and columns,
 * in increasing index order (gke_sample_indices).  Before gke_set_workspace.
 * Errors: GKE_ERR_ARG (dir, t1 < 0, t2 < t1, a step < 1), GKE_ERR_STATE. */
gke_status gke_set_undersampling(gke_plan_t plan, int dir, int t1, int t2, int s1, int s2);

/* Kept grid indices of the output maps along rx (dir 0: among 0..Nx/2 in the
 * ALLPAIRS_HALFRX domain, 0..Nx-1 in the full-r domains) or rz (dir 1, among
 * 0..Nz-1), increasing: *count receives their number and idx, when not NULL,
 * the indices (host array of at least Nx or Nz ints).  Follows the options in
 * effect.  Errors: GKE_ERR_ARG, and those of gke_workspace_size. */
gke_status gke_sample_indices(gke_plan_t plan, int dir, int *count, int *idx);

/* Device workspace bytes the plan needs with its current options (fixes the
 * automatic chunk).  Errors: GKE_ERR_ARG (NULL; the fundamental domain without
 * the mirror), GKE_ERR_UNSUPPORTED (the spectra of one kx wavenumber reach
 * 2^31 elements, Nz * 10 * chunk * Ny rounded up; split-BF16 with Nz above
 * 972, whose four-snapshot z transforms exceed one block's LDS). */
gke_status gke_workspace_size(gke_plan_t plan, size_t *bytes);

/* Hand the plan a caller-owned device buffer of at least gke_workspace_size
 * bytes (256-byte aligned).  The caller keeps ownership and must keep it
 * alive until gke_destroy.  Fixes the options.  Errors: GKE_ERR_OOM if too
 * small, GKE_ERR_ARG for NULL/misaligned, GKE_ERR_STATE if already set, and
 * those of gke_workspace_size. */
gke_status gke_set_workspace(gke_plan_t plan, void *device_ptr, size_t bytes);

/* Size of the library-owned workspace of gke_set_static_workspace. */
#define GKE_STATIC_WORKSPACE_BYTES ((size_t)64 << 20)

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same as
 * gke_set_workspace, but the plan takes the library's own static device
 * workspace of GKE_STATIC_WORKSPACE_BYTES instead of a caller buffer.  Set the
 * stream (gke_set_stream) first: the tables are uploaded and the sums cleared
 * on it.  The call allocates nothing (no hipMalloc, hipFree or allocating
 * library routine); inputs and outputs are still the caller's.
 * Sharing: there is one static workspace per GPU, that of the device current
 * at this call, held until the process ends; the plan must run on that
 * device.  Every plan that takes it on one GPU uses the same memory, which
 * keeps the last plan's contents: this call re-uploads the tables and clears
 * what must start at zero, so plans used one after another are independent,
 * but plans whose work overlaps on one GPU race (use one at a time).
 * Errors: GKE_ERR_OOM (the plan, with its options, needs more than
 * GKE_STATIC_WORKSPACE_BYTES: see gke_workspace_size), GKE_ERR_STATE (a
 * workspace is already set), GKE_ERR_HIP (device or symbol lookup failed),
 * and those of gke_workspace_size. */
gke_status gke_set_static_workspace(gke_plan_t plan);

/* HIP stream (hipStream_t) on which all work is enqueued; NULL = default. */
gke_status gke_set_stream(gke_plan_t plan, void *hip_stream);

/* Add one snapshot: device pointers to u~, v~, w~, p~ ([Ny][Nz][Nx], the
 * plan's dtype).  Before gke_begin_stats the call belongs to the first scan
 * (sums for the means); afterwards to the second scan (two-point statistics).
 * Asynchronous; the library does not keep the pointers once the enqueued work
 * has run, so the caller may reuse the buffers after a stream synchronisation.
 * Errors: GKE_ERR_ARG (NULL), GKE_ERR_STATE (no workspace), GKE_ERR_HIP. */
gke_status gke_accumulate(gke_plan_t plan, const void *u, const void *v, const void *w,
                          const void *p);

/* Step 1 upstream of the statistics (Section "Step 1": a database holding the
 * wall-normal velocity and vorticity as Fourier coefficients; the full
 * velocity is computed and the pressure obtained from its Poisson equation).
 * In: vhat, ohat, device complex FP64 (re, im interleaved, 16-byte aligned) coefficients of v
 * and omega_y = du/dz - dw/dx, layout [Ny][Nz][Nx/2 + 1], f(x, z) =
 * sum_k f^ e^{i(alpha x + beta z)} over the half spectrum (the forward
 * transform divided by Nx Nz); mean_u, mean_w, device FP64 [Ny], the (0, 0)
 * coefficients of u and w.  Out: device FP64 u, v, w, p [Ny][Nz][Nx] (the
 * layout gke_accumulate reads with GKE_DTYPE_F64).  alpha = 2 pi kx/Lx and
 * beta = 2 pi kz/Lz are 0 at the Nyquist wavenumbers.
 *   velocity, k^2 = alpha^2 + beta^2 > 0 (continuity and the definition of
 *     omega_y):  u^ = i (alpha D v^ - beta omega^)/k^2,
 *                w^ = i (beta D v^ + alpha omega^)/k^2;
 *   pressure: lap p = -d_i d_j (u_i u_j) with the total velocity (products on
 *     the grid), per wavenumber (D2 - k^2) p^ = alpha^2 uu^ + 2 alpha beta uw^
 *     + beta^2 ww^ - 2 i alpha D uv^ - 2 i beta D vw^ - D2 vv^ at the interior
 *     nodes, D p^ = nu D2 v^ at the two walls (wall-normal momentum with no
 *     slip), solved per wavenumber by banded elimination with partial
 *     pivoting; the (0, 0) coefficient p^ = -vv^ (the mean pressure does not
 *     enter the terms) and 0 in the other bins with k^2 = 0;
 *   D: the five-point first derivative used everywhere; D2: the five-point
 *     second-derivative weights on the same node windows.
 * Needs GKE_OPT_STEP1 = 1 before the workspace (about 19 Ny Nk complex FP64
 * values more).  Asynchronous on the plan's stream; reads nothing else of the
 * plan's state, so it may be called before or between gke_accumulate calls.
 * Errors: GKE_ERR_ARG (NULL, vhat or ohat not 16-byte aligned), GKE_ERR_STATE
 * (no workspace, option not set), GKE_ERR_HIP. */
gke_status gke_reconstruct(gke_plan_t plan, const void *vhat, const void *ohat,
                           const double *mean_u, const double *mean_w, double *u, double *v,
                           double *w, double *p);

/* The same as n calls of gke_accumulate with u[i], v[i], w[i], p[i] (host
 * arrays of n device pointers), launched as one HIP graph: the launches are
 * captured once (on a stream of the library's own) and the executable graph
 * is replayed on the plan's stream as long as the pointers, n and the scan
 * state at the call (which scan, the position in the current chunk) match; a
 * different batch re-captures and updates the graph in place (up to four are
 * kept per plan).  With GKE_OPT_TIMING the launches are made one by one.
 * Errors: those of gke_accumulate, GKE_ERR_HIP for capture or launch. */
gke_status gke_accumulate_batch(gke_plan_t plan, int n, const void *const *u,
                                const void *const *v, const void *const *w,
                                const void *const *p);

/* Close the first scan: means U V W P from the snapshots accumulated so far
 * and S = dU/dy.  Errors: GKE_ERR_STATE if no snapshot was accumulated or
 * the second scan already started. */
gke_status gke_begin_stats(gke_plan_t plan);

/* Alternative to the first scan: host FP64 means U, V, W, P of length Ny.
 * Errors: GKE_ERR_ARG (NULL), GKE_ERR_STATE (second scan already started). */
gke_status gke_set_means(gke_plan_t plan, const double *U, const double *V, const double *W,
                         const double *P);

/* Average, inverse transforms, assembly and the five-point derivatives; write
 * the requested maps (see gke_terms).  Blocking for device outputs; with host
 * outputs it returns once the maps are in the staging buffer and their copies
 * are enqueued (gke_wait_outputs).  Does not consume the plan:
 * more snapshots may be accumulated and finalize called again.  Errors:
 * GKE_ERR_STATE (no second-scan snapshot, or the two scans have different
 * snapshot counts; host outputs without staging; the residual without
 * GKE_OPT_RESIDUAL), GKE_ERR_ARG (dtype; a map the requested terms need is
 * missing), GKE_ERR_UNSUPPORTED (the residual in the slab modes), GKE_ERR_HIP. */
gke_status gke_finalize(gke_plan_t plan, const gke_terms *out);

/* Checkpoint and resume of the accumulation (the paper's program keeps its
 * running sums on disk and divides them only at the end, Section "General
 * structure of the program": a long scan can stop and continue).  The state
 * is the scan counters, the one-point sums and moment partials, the
 * cross-spectral accumulators and, in the general modes, the band
 * accumulators, with a header naming the plan's shape and options.
 * gke_state_size: the bytes of the state (it grows with the accumulators:
 * 8 * Nk * pairs * 16 bytes, 18.6 GB at Re_tau=200).
 * gke_save_state: first adds the snapshots of the current chunk into the
 * accumulators (as gke_finalize does), then copies the state into `host`
 * (caller-owned host memory, pageable or pinned, at least gke_state_size
 * bytes); blocking.  The plan continues unchanged afterwards.
 * gke_load_state: replaces the scan state of a plan with a workspace by a
 * saved one; the plan must have the same grid, y, Lx, Lz, nu, dtype,
 * precision, mirror, domain, slab rows and undersampling (chunk and block
 * shapes may differ); in the general modes it selects the saved slab.
 * Blocking.  The continued run equals the uninterrupted one with the same
 * chunk boundaries bit for bit.
 * Errors: GKE_ERR_ARG (NULL, buffer too small, not a saved state, another
 * shape or options), GKE_ERR_STATE (no workspace), GKE_ERR_HIP. */
gke_status gke_state_size(gke_plan_t plan, size_t *bytes);
gke_status gke_save_state(gke_plan_t plan, void *host, size_t bytes);
gke_status gke_load_state(gke_plan_t plan, const void *host, size_t bytes);

/* Notification per slab (Section "Undersampling and parallelisation": the
 * wall-normal slices are computed one after another, each slice's results
 * written out as it completes).  fn(slab, user) is called once per
 * gke_finalize, on a HIP runtime thread, once that finalize's maps are
 * complete where the caller reads them: for host outputs after the copies to
 * the host arrays (so a caller may consume or reuse a slab's host arrays
 * there, while the next slab scans), for device outputs after the kernels.
 * slab is the slab being finalized (0 in the all-pairs mode).  fn must return
 * promptly and must not call HIP or any gke_ function (the stream it runs on
 * waits for it); fn = NULL removes the notification.  Allowed at any time;
 * the plan keeps fn and user, the caller owns what user points to.
 * Errors: GKE_ERR_ARG (NULL plan); a failure to enqueue the call is reported
 * by gke_finalize (GKE_ERR_HIP). */
typedef void (*gke_slab_fn)(int slab, void *user);
gke_status gke_set_slab_callback(gke_plan_t plan, gke_slab_fn fn, void *user);

/* Wait until the host copies of every gke_finalize with host outputs have
 * completed (returns at once when there are none).  Errors: GKE_ERR_ARG,
 * GKE_ERR_HIP. */
gke_status gke_wait_outputs(gke_plan_t plan);

/* Number of slabs (after gke_set_workspace): 1 unless GKE_OPT_SLAB cuts the
 * output rows.  Errors: GKE_ERR_STATE (no workspace). */
gke_status gke_slab_count(gke_plan_t plan, int *count);

/* Output pairs of slab `slab` in layout order: *count receives their number
 * and, when pairs is not NULL, pairs[2 n] = Y1 index, pairs[2 n + 1] = Y2
 * index (host array of 2 * count ints).  Errors: GKE_ERR_ARG, GKE_ERR_STATE. */
gke_status gke_slab_pairs(gke_plan_t plan, int slab, int *count, int *pairs);

/* Start the second scan of slab `slab` (after gke_begin_stats or
 * gke_set_means, which start slab 0): forgets the second-scan snapshots of
 * the previous slab; the caller then accumulates every snapshot again and
 * calls gke_finalize for this slab's maps.  Enqueued on the plan's stream.
 * Errors: GKE_ERR_ARG (slab out of range), GKE_ERR_STATE (means not known). */
gke_status gke_begin_slab(gke_plan_t plan, int slab);

/* Copy the GKE_NPROF x Ny profile block (row-major, FP64) to host memory
 * `out`.  Valid after gke_finalize (rows U..S after gke_begin_stats). */
gke_status gke_get_profiles(gke_plan_t plan, double *out);

/* Forget every accumulated snapshot (both scans) so that the same plan and
 * workspace start a new ensemble; enqueued on the plan's stream.
 * Errors: GKE_ERR_STATE (no workspace), GKE_ERR_HIP. */
gke_status gke_reset(gke_plan_t plan);

/* kernel families reported by gke_timings (GKE_K_RANKK: the matrix-core
 * update of full 16-plane tiles; GKE_K_RANKK_REM: the pairs that involve the
 * last Ny mod 16 planes; GKE_K_RESID: the two residual passes, the kz
 * transform of its spectral divergence and its five-point Y part;
 * GKE_K_STEP1: one gke_reconstruct, all its launches) */
enum { GKE_K_PLANE_SUMS = 0, GKE_K_FLUCT_XFFT, GKE_K_ZFFT_PACK, GKE_K_RANKK, GKE_K_FIN_KZ,
       GKE_K_FIN_KX, GKE_K_FD, GKE_K_SMALL, GKE_K_RANKK_REM, GKE_K_RESID, GKE_K_STEP1,
       GKE_NKERNELS };

/* With GKE_OPT_TIMING set, HIP events bracket every kernel launch on the
 * plan's stream.  Synchronises the stream, then writes per kernel family the
 * summed device time in milliseconds (total_ms[GKE_NKERNELS]) and the number
 * of launches (launches[GKE_NKERNELS]) since the last reset of the counters;
 * reset != 0 clears them.  Either output may be NULL. */
gke_status gke_timings(gke_plan_t plan, double *total_ms, int64_t *launches, int reset);

/* Release the plan (synchronises its stream; never frees the workspace). */
void gke_destroy(gke_plan_t plan);

/* Text of the last error on `plan` (or of the last failed gke_plan when
 * plan is NULL).  The string lives until the next call on the plan. */
const char *gke_last_error(gke_plan_t plan);

/* Library version string. */
const char *gke_version(void);

#ifdef __cplusplus
}
#endif
#endif /* GKE_H */
