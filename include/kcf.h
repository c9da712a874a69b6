/*
 * kcf.h — C ABI of the MI355X (gfx950) library for explicit filtering, Favre filtering,
 * subgrid-scale (SGS) tensors, closure expressions and a learned SGS closure on periodic
 * 3-D grids.
 *
 * The quantities follow the definitions of the kinetic-closure paper (Marson & Malaspinas,
 * "Kinetic closure of turbulence: collision-side modeling beyond the filtered Boltzmann
 * equation"):
 *   - homogeneous LES filter bar(.) of uniform width Delta (Sec. "Filtered nondimensional
 *     recorrelated BGK-BE"; the kernel shape is not prescribed there, so the library offers
 *     a trapezoidal box and a truncated Gaussian, see kcf_filter_taps);
 *   - Favre velocity ut_i = bar(rho u_i) / bar(rho) (definition after eq. f0resolved);
 *   - SGS second moment tau_ij = m^sgs_ij = bar(rho u_i u_j) - rho_bar ut_i ut_j (eq. m_sgs_2);
 *   - velocity gradient by central differences (App. "Lattice-Boltzmann discretization",
 *     eqs. fd and strain_rate_discrete);
 *   - closure expressions: tensor-diffusivity (gradient) model (eq. ansumali), eddy
 *     viscosity of the Boussinesq row of the FNSE/FRBGK comparison table with the
 *     Smagorinsky constant of Sec. "Test cases", and the kinetic-closure scalars k_sgs, nu_t,
 *     omega_t (Sec. "Turbulent relaxation frequency", eqs. ksgs_sharp_trace,
 *     nu_t_sharp_closure, omega_t_sharp_closure; operational eq. omega_sgs_operational);
 *   - volume averages of eq. tgv_energy_enstrophy.
 *
 * Conventions for every entry point
 *   Fields are float32, contiguous, structure-of-arrays, x fastest: point (i, j, k) of an
 *   nx*ny*nz grid is element i + nx*(j + ny*k). A vector field is 3 consecutive blocks
 *   (x|y|z); a symmetric tensor is 6 blocks in the order xx xy xz yy yz zz; the gradient is
 *   9 blocks G_ij = d_j ut_i in row-major order (xx xy xz yx yy yz zx zy zz).
 *   The grid is periodic in all directions with uniform spacing h.
 *   Field pointers are DEVICE pointers owned by the caller; the library never frees them.
 *   Structs of parameters and statistics are HOST memory.
 *   Work is enqueued on the context's HIP stream. Calls that return host statistics
 *   synchronise that stream before returning; the others are asynchronous.
 *   Every call returns a kcf_status; no call aborts or throws across the ABI. On failure
 *   kcf_last_error() gives a message (per thread).
 */
#ifndef KCF_H
#define KCF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  KCF_OK = 0,
  KCF_EINVAL = -1,        /* invalid argument (null pointer, bad size, odd box width, ...) */
  KCF_ENOMEM = -2,        /* device allocation failed */
  KCF_EHIP = -3,          /* HIP runtime error */
  KCF_EUNSUPPORTED = -4,  /* valid request the GPU path does not support (e.g. 2R+1 > n) */
  KCF_EIO = -5            /* file error (checkpoints) */
} kcf_status;

typedef enum { KCF_BOX = 0, KCF_GAUSS = 1 } kcf_kind;

typedef struct kcf_ctx kcf_ctx;
typedef struct kcf_mlp kcf_mlp;

typedef struct { int nx, ny, nz; double h; } kcf_grid;

/* kind: KCF_BOX (delta_over_h even, >= 2) or KCF_GAUSS (delta_over_h >= 1).
 * precision of the filter sums and of the Favre/tau assembly: 0 = auto (FP64 for widths up
 * to 4h, where tau is a small difference of large filtered products, FP32 above), 1 = FP32,
 * 2 = FP64. Outputs are float32 in every case. */
typedef struct { int kind; int delta_over_h; int precision; } kcf_filter;

/* Device output buffers of one filter width; any pointer may be NULL (not produced). */
typedef struct {
  float *rho_bar;   /* N   */
  float *ut;        /* 3N  */
  float *tau;       /* 6N  */
  float *grad;      /* 9N  */
  float *tau_gm;    /* 6N  gradient model */
  float *tau_smag;  /* 6N  deviatoric eddy-viscosity model */
  float *k_sgs;     /* N   */
  float *nu_t;      /* N   */
  float *omega_t;   /* N   */
  float *q_crit;    /* N   Q-criterion (|W|^2 - |S|^2)/2 of the gradient (W, S its antisymmetric
                           and symmetric parts), the vortex indicator of the paper's cavity
                           and cylinder sections */
} kcf_outputs;

/* Closure parameters. Pass NULL for the defaults given in brackets. */
typedef struct {
  double c_s;        /* Smagorinsky constant [0.11] */
  double c_nu;       /* kinetic-closure constant C_nu [0.02] */
  double theta;      /* reference temperature theta (c_s^2 in velocity units) [1] */
  double nu_mol;     /* molecular viscosity for the clip min(omega, omega_t) [0: none] */
  double dt;         /* time step of the shifted rate (nu/theta + dt/2)^-1 [0: continuum] */
  int gm_form;       /* 0: tau_gm = rho_bar C2 G G^T (Taylor) [0]; 1: rho_bar C2 G^T G */
  int m2_mode;       /* 0: C2 = second moment of the discrete kernel [0]; 1: Delta^2/12 */
  int ksgs_rho_ref;  /* 0: k_sgs = |tau_kk|/(2 rho_bar) [0]; 1: |tau_kk|/2 (rho0 = 1) */
} kcf_closure_params;

/* FP64 statistics of one filter width (global reductions on the GPU). Box widths up to 8h
 * with precision 2 (FP64 requested explicitly) form each point's contributions as exact FP64
 * products of its float32 outputs. Every other width (precision 0 or 1, and the general-tap
 * path's closure pass at any precision) forms them in float32 and sums at most 16 points
 * (64 contributions: over four lanes per point where the filter sums are FP64, per lane
 * where they are float32) in float32 before the FP64 reduction: a raw sum is then within
 * 25 * 2^-24 of the sum of its terms' magnitudes, about the rounding of the float32 outputs
 * themselves. A point with a non-finite contribution (a non-finite output, or a float32
 * product beyond range) is counted in n_nonfinite. */
typedef struct {
  double delta, m2;             /* filter width, second moment of the discrete kernel */
  double mean_rho_bar;          /* <rho_bar> */
  double ke_resolved;           /* <rho_bar |ut|^2 / 2> */
  double pi;                    /* SGS dissipation -<tau_ij S_ij> */
  double pi_gm;                 /* -<tau_gm_ij S_ij> */
  double pi_smag;               /* -<tau_smag_ij S_ij> */
  double corr_tau_gm[6];        /* Pearson r(tau_c, tau_gm_c), c = xx xy xz yy yz zz */
  double corr_pi;               /* Pearson r(-tau:S, -tau_gm:S) over points */
  double mean_tau[6];
  int64_t n_points;             /* points counted (finite outputs) */
  int64_t n_nonfinite;          /* points with a non-finite output (excluded from sums) */
  double raw[40];               /* the raw FP64 sums the above are derived from */
} kcf_width_stats;

/* Statistics of the SGS carrier (kcf_sgs_carrier), means over the finite points: each
 * point's sums over its 27 populations in FP32, their sums over points in FP64. */
typedef struct {
  double sgs_l2;                /* <sum_i f_sgs,i^2> */
  double err_l2;                /* <sum_i (f_sgs,i - f_h2,i)^2> */
  double rel_err;               /* sqrt(err_l2 / sgs_l2): relative L2 error of f_h2 */
  double hermite[5];            /* <E_n>, n = 2..6: weighted energy sum_i f_i^2 / w_i of the
                                   Hermite terms of order n (E_0 = E_1 = 0 exactly) */
  int64_t n_points;             /* points counted (finite outputs) */
  int64_t n_nonfinite;          /* points with a non-finite output (excluded from sums) */
  double raw[9];                /* the raw FP64 sums: count, sum f^2, sum (f - f_h2)^2,
                                   E_2..E_6, non-finite count */
} kcf_carrier_stats;

/* Statistics of the third-order SGS moment (kcf_sgs_moment3), over the finite points; the
 * components in the order xxx xxy xxz xyy xyz xzz yyy yyz yzz zzz. */
typedef struct {
  double mean_m3[10];           /* <m3_c> */
  double rms_m3[10];            /* sqrt(<m3_c^2>) */
  double mean_theta_t;          /* <theta_t> (1 without a temperature field) */
  int64_t n_points;             /* points counted (finite outputs) */
  int64_t n_nonfinite;          /* points with a non-finite output (excluded from sums) */
  double raw[23];               /* count, sums of m3_c, sums of m3_c^2, sum of theta_t,
                                   non-finite count */
} kcf_moment3_stats;

/* Parameters of the KC-MP evaluation (kcf_kc_mp). */
typedef struct {
  double nu;          /* molecular kinematic viscosity (>= 0), in the units of u and h */
  double dt;          /* time step of the shifted relaxation time tau_hat = nu/theta + dt/2
                         (>= 0; 0 = continuum) */
  double theta;       /* reference temperature theta_R (> 0; c_s^2 in the units of u) */
  double c_nu;        /* closure constant C_nu (the paper's KC-MP value is 0.035) */
  int rho_ref_one;    /* 1: k_sgs = |m_aa| / 2 (operational reference density 1);
                         0: |m_aa| / (2 rho_bar) */
} kcf_kc_params;

/* Statistics of the KC-MP evaluation against the exact tau, over the finite points. */
typedef struct {
  double corr[6];               /* Pearson r(m_sgs_c, tau_c), c = xx xy xz yy yz zz */
  double rel_err;               /* (sum |m_sgs - tau|_F^2 / sum |tau|_F^2)^(1/2), all 9 pairs */
  double mean_m[6], mean_tau[6];
  double mean_k, mean_k_exact;  /* <k_sgs> from m_sgs and from tau */
  double mean_omega, mean_omega_exact;  /* <omega_sgs> from m_sgs and from tau */
  double clip, clip_exact;      /* fraction of points with nu_t_eff = nu */
  int64_t n_points, n_nonfinite;
  double raw[40];               /* the raw FP64 sums */
} kcf_kc_stats;

typedef struct {
  double mean_rho;              /* <rho> */
  double ek;                    /* <rho |u|^2 / 2> */
  double enstrophy;             /* <|curl u|^2 / 2>, sixth-order central differences */
  int64_t n_nonfinite;
} kcf_input_summary;

/* ---- library and context ------------------------------------------------------------ */
int kcf_version(void);  /* 10000 * major + 100 * minor + patch */

/* Create a context on HIP device `device` that enqueues on `stream` (hipStream_t, NULL =
 * default stream). The context owns its scratch memory: the FP64 partial sums of the
 * reductions and, grown on demand and kept until kcf_ctx_destroy, the slab and field buffers
 * of the multi-kernel paths. */
int kcf_ctx_create(kcf_ctx **out, int device, void *stream);
int kcf_ctx_set_stream(kcf_ctx *ctx, void *stream);
void kcf_ctx_destroy(kcf_ctx *ctx);
const char *kcf_last_error(void);

/* Kernel timing: when enabled, every launch of the filter kernel is bracketed by HIP events
 * on the context stream; kcf_ctx_kernel_ms returns the summed time of the launches since
 * the last reset (and the number of launches) after synchronising the stream. */
int kcf_ctx_enable_timing(kcf_ctx *ctx, int on);
int kcf_ctx_kernel_ms(kcf_ctx *ctx, double *ms, int *launches);
/* The same record launch by launch: ms[i] (host, cap entries) is the time of the i-th timed
 * launch since the last reset, in launch order (a call of kcf_filter_favre launches one
 * kernel per width, in the order of its filters). KCF_EINVAL if cap is too small. Resets. */
int kcf_ctx_kernel_times(kcf_ctx *ctx, float *ms, int cap, int *launches);

/* ---- host helper (no GPU) ------------------------------------------------------------ */
/* 1-D taps w_{-R..R} of the filter used by the GPU (float32), its radius R and the second
 * moment M2 = sum w_m (m h)^2 computed in double. box: R = n/2, w = 1/n inside and 1/(2n)
 * at the ends (trapezoidal top-hat of width n h). gauss: exp(-6 m^2/n^2) for |m| <=
 * ceil(1.5 n), normalised to unit sum. `cap` is the capacity of w (2R+1 needed). */
int kcf_filter_taps(int kind, int delta_over_h, double h, float *w, int cap, int *radius,
                    double *m2);

/* ---- the filtering path --------------------------------------------------------------- */
/* For each of n_filters (1..4) widths, one kernel launch, in one pass over rho (N) and u (3N):
 * products rho, rho u_i, rho u_i u_j; separable periodic filter; Favre division;
 * tau; central-difference gradient of ut; closures; FP64 statistics.
 * outs[f] selects the fields written for width f (NULL members are skipped). stats may be
 * NULL; when given it has n_filters entries, the gradient, both closures and the statistics
 * are evaluated on chip, and the call synchronises the stream. Without stats the gradient
 * and closures are evaluated only for the fields outs[f] asks for (none for rho_bar, ut and
 * tau alone).
 * Box widths up to 16h (FP32) or 8h (FP64) run as one fused kernel per width. Other widths
 * (Gaussian, wider box) run as an x-y pass into a context buffer of filtered products (the
 * whole field or z slabs; 8 GiB, raised up to 48 GiB while half of the free device memory
 * stays free; the outputs do not depend on the slab count), a z pass writing rho_bar, ut, tau, and,
 * when the gradient is needed, the pass of kcf_grad_closure on those fields; if the caller
 * does not ask for rho_bar, ut or tau the context holds them in a scratch of 10 N floats.
 * Errors: KCF_EINVAL for null rho/u/outs/grid, n < 3 in any direction, n_filters outside
 * 1..4, bad filter kind or width; KCF_EUNSUPPORTED when 2R+1 exceeds a grid dimension,
 * R > 12 or ny > 65535; KCF_ENOMEM when a context buffer cannot be allocated. */
int kcf_filter_favre(kcf_ctx *ctx, const kcf_grid *grid, const kcf_filter *filters,
                     int n_filters, const float *rho, const float *u, const kcf_outputs *outs,
                     const kcf_closure_params *cp, kcf_width_stats *stats);

/* The box path of kcf_filter_favre for callers that cannot allocate device memory (code under
 * HIP graph capture, serving loops, harnesses that forbid hipMalloc): the same kernels and
 * results, with no context. Work is enqueued on `stream` (hipStream_t, NULL = default stream)
 * of HIP device `device`. The call allocates nothing: its FP64 statistics records, reduction
 * totals and sums live in a 16 MiB device array of the library that each GPU holds for the life
 * of the process. Every call on a GPU shares that array, so calls that overlap on one GPU (on
 * different streams or host threads) race and must be serialised by the caller. Without stats
 * the array is not used and the call is asynchronous; with stats it synchronises the stream.
 * Limits: box filters only (widths up to 16h in FP32, 8h in FP64); with stats, at most
 * 52 168 statistics records per width (one per wave of the box kernel: a 512^3 grid needs at
 * most 27 520; 1024^3 grids exceed it at the narrow widths).
 * Errors: as kcf_filter_favre; KCF_EUNSUPPORTED for a Gaussian or wider box filter and for a
 * grid whose records exceed the array, KCF_EINVAL for a bad device index. */
int kcf_filter_favre_noalloc(const kcf_grid *grid, const kcf_filter *filters, int n_filters,
                             const float *rho, const float *u, const kcf_outputs *outs,
                             const kcf_closure_params *cp, kcf_width_stats *stats, int device,
                             void *stream);

/* Gradient, closures and statistics from stored filtered fields rho_bar (N), ut (3N) and
 * tau (6N, may be NULL: then k_sgs/nu_t/omega_t and tau statistics are not available and
 * must not be requested). delta = filter width, m2 = kernel second moment. */
int kcf_grad_closure(kcf_ctx *ctx, const kcf_grid *grid, const float *rho_bar, const float *ut,
                     const float *tau, double delta, double m2, const kcf_closure_params *cp,
                     const kcf_outputs *outs, kcf_width_stats *stats);

/* A priori SGS carrier of the D3Q27 lattice for one filter width: the residual
 *   f_sgs,i = bar(f0_i(rho, u)) - f0_i(rho_bar, ut)
 * of filtering the equilibrium (Sec. "Filtered nondimensional recorrelated BGK-BE",
 * eqs. f0bar and fsgs_def), with the product equilibrium of App. "Lattice-Boltzmann
 * discretization" (eq. discrete_equilibrium), and its second-order Hermite reconstruction
 *   f_h2,i = w_i / 2 (xh_ia xh_ib - delta_ab) tau_ab
 * of the KC-MP closure (Sec. "Moment-Projected Closure (KC-MP)", eq. f_sgs_KCMP).
 * Units: velocities u in units of sqrt(theta_R) (Mach numbers); xh_i = xi_i / sqrt(theta_R) in
 * {0, +-sqrt(3)}^3 for the lattice velocities xi_i in {-1, 0, 1}^3; w_i = product of the D1Q3
 * weights 2/3 (0) and 1/6 (+-1); populations in units of density. Population i is
 * xi_i = (c_x, c_y, c_z) with i = 9 (c_x + 1) + 3 (c_y + 1) + (c_z + 1).
 * f_sgs and f_h2 (device, 27 N floats each, population blocks [i][N]) and stats (host) may
 * each be NULL, but not all three. filter->precision as for kcf_filter_favre (auto: FP64 for
 * widths up to 4h). The call filters the 27 monomials rho u_x^a u_y^b u_z^c (a, b, c <= 2)
 * in z slabs through a context buffer of at most 8 GiB and launches two kernels per slab
 * (both timed when timing is on); with stats it synchronises.
 * Errors: KCF_EINVAL for null rho/u/grid/filter, nothing requested, bad filter or n < 3;
 * KCF_EUNSUPPORTED when 2R+1 exceeds a grid dimension, R > 12 or ny > 65535; KCF_ENOMEM when a
 * context buffer cannot be allocated. */
int kcf_sgs_carrier(kcf_ctx *ctx, const kcf_grid *grid, const kcf_filter *filter,
                    const float *rho, const float *u, float *f_sgs, float *f_h2,
                    kcf_carrier_stats *stats);

/* Third-order SGS moment and Favre temperature for one filter width:
 *   m3_ijk  = bar(rho u_i u_j u_k) - rho_bar ut_i ut_j ut_k   (10 components, device [10][N],
 *             order xxx xxy xxz xyy xyz xzz yyy yyz yzz zzz),
 * the coefficient of the third-order Hermite term of the carrier's series (Sec. "Filtered
 * nondimensional recorrelated BGK-BE", eq. f_sgs_hermite; with the same velocity units as
 * kcf_sgs_carrier), and
 *   theta_t = bar(rho theta) / rho_bar                        (device [N]),
 * the Favre temperature (definition after eq. f0resolved). theta (device [N]) may be NULL
 * (isothermal: then theta_t must be NULL and its statistic is 1). m3, theta_t and stats (host)
 * may each be NULL, but not all three. filter->precision as for kcf_filter_favre. The call
 * filters 14 quantities (15 with theta) in z slabs through a context buffer of at most
 * 8 GiB, two timed kernels per slab; with stats it synchronises.
 * Errors: KCF_EINVAL for null rho/u/grid/filter, nothing requested, theta_t without theta,
 * bad filter or n < 3; KCF_EUNSUPPORTED when 2R+1 exceeds a grid dimension, R > 12 or
 * ny > 65535; KCF_ENOMEM when a context buffer cannot be allocated. */
int kcf_sgs_moment3(kcf_ctx *ctx, const kcf_grid *grid, const kcf_filter *filter,
                    const float *rho, const float *u, const float *theta, float *m3,
                    float *theta_t, kcf_moment3_stats *stats);

/* A priori evaluation of the KC-MP closure for one filter width (App. "Operational
 * implementation of KC-MP", Sec. "Moment-Projected Closure (KC-MP)"). The fine-grained state
 * is taken as f0(rho, u) plus its Chapman-Enskog part, whose second moment is
 * -2 rho theta tau_hat S(u) (S from the central differences of eqs. fd and
 * strain_rate_discrete); filtering it gives the coarse non-equilibrium moment
 * m_cneq = tau - 2 theta tau_hat bar(rho S), and the closure's SGS moment is
 *   m_sgs = m_cneq - m_CE = tau - 2 theta tau_hat (bar(rho S) - rho_bar S_t),
 * m_CE = -2 rho_bar theta tau_hat S_t, S_t = S(ut) (eq. m_ce_reference and its operational
 * form). From m_sgs, the relaxation-rate field of eq. omega_sgs_operational:
 *   k_sgs = |m_sgs_aa| / (2 rho_ref), nu_t_eff = max(nu, C_nu Delta sqrt(k_sgs)),
 *   omega_sgs = (nu_t_eff / theta + dt / 2)^-1     (Delta = the filter width),
 * and the same rates from the exact tau for the statistics. Outputs (device, each may be
 * NULL, but not all of them and stats): m_sgs and m_ce [6][N] (xx xy xz yy yz zz), k_sgs,
 * nu_t_eff, omega_sgs [N]. The call runs the filter path (kcf_filter_favre, into a context scratch of
 * 16 N floats for rho_bar, tau and G), then filters rho S_ij in z slabs (two timed kernels
 * per slab); with stats it synchronises.
 * Errors: as kcf_sgs_carrier; KCF_EINVAL for a NULL or out-of-range kp. */
int kcf_kc_mp(kcf_ctx *ctx, const kcf_grid *grid, const kcf_filter *filter, const float *rho,
              const float *u, const kcf_kc_params *kp, float *m_sgs, float *m_ce, float *k_sgs,
              float *nu_t_eff, float *omega_sgs, kcf_kc_stats *stats);

/* ---- D3Q27 lattice-Boltzmann solver with the kinetic closures -------------------------
 * One collide-and-stream step of the paper's solver (App. "Lattice-Boltzmann discretization"
 * and App. "Common operational algorithm") on a periodic lattice, in lattice units
 * (Delta x = Delta t = 1, lattice velocities xi_i in {-1, 0, 1}^3, theta_R = 1/3; grid->h is
 * not used). Populations are the time-shifted populations of eq.
 * shifted_population_definition, float32 [27][N] blocks in the population order of
 * kcf_sgs_carrier (i = 9 (c_x + 1) + 3 (c_y + 1) + (c_z + 1)).
 * Per node: rho = sum_i f_i, rho u = sum_i f_i xi_i; the product equilibrium f0 (eq.
 * discrete_equilibrium); S from central differences of u (eqs. fd, strain_rate_discrete);
 * the closure's SGS trace; k_sgs = |m_aa| / 2 (reference density 1), nu_t_eff =
 * max(nu, C_nu sqrt(k_sgs)) (Delta = Delta x), omega_sgs = (nu_t_eff / theta_R + 1/2)^-1
 * (eq. omega_sgs_operational); omega = (nu / theta_R + 1/2)^-1 (eq. omega_t_discrete); the
 * collision of the model; streaming f_i(x + xi_i, t + 1) = f_post_i(x, t) (eq. streaming). */
typedef enum {
  KCF_LBM_BGK = 0,       /* resolved BGK: f_post = f - omega (f - f0) */
  KCF_LBM_KCRB = 1,      /* KC-RB, Hermite first-order part (eqs. kcrb_operational_fone,
                            kcrb_operational_msgstrace, kcrb_operational_collision) */
  KCF_LBM_KCRB_RAW = 2,  /* KC-RB with the raw xi xi first-order part of the paper's runs
                            (eq. kcrb_operational_raw_fone) */
  KCF_LBM_KCMP = 3,      /* KC-MP (eqs. kcmp_operational_msgstrace, kcmp_operational_collision) */
  KCF_LBM_KCRR = 4       /* KC-RR (eqs. kcrr_operational_second_order_collision,
                            kcrr_operational_high_order_collision,
                            kcrr_operational_post_population, RR recursion eq. kcrr_rr) */
} kcf_lbm_model;

typedef struct {
  int model;     /* kcf_lbm_model */
  double nu;     /* molecular kinematic viscosity, lattice units (> 0) */
  double c_nu;   /* closure constant C_nu (>= 0; the paper uses 0.02 for KC-RB and KC-RR,
                    0.035 for KC-MP); 0 makes every closure the BGK step */
} kcf_lbm_params;

/* FP64 sums over the nodes of the state entering the step (reduced on the GPU). */
typedef struct {
  double mass;             /* sum rho */
  double momentum[3];      /* sum rho u */
  double kinetic_energy;   /* sum rho |u|^2 / 2 */
  double mean_omega_sgs;   /* <omega_sgs> (omega for BGK) */
  double clip_fraction;    /* fraction of nodes with C_nu sqrt(k_sgs) <= nu (1 for BGK) */
  double mean_k_sgs;       /* <k_sgs> */
  int64_t n_nodes;
  double raw[8];           /* the raw sums */
} kcf_lbm_stats;

/* Equilibrium populations f_out [27][N] of density rho [N] and velocity u [3][N] (lattice
 * units), e.g. to start a run. Asynchronous. Errors: KCF_EINVAL for NULL arguments or a bad
 * grid. */
int kcf_lbm_equilibrium(kcf_ctx *ctx, const kcf_grid *grid, const float *rho, const float *u,
                        float *f_out);

/* One time step from f_in to f_out (distinct device buffers [27][N], both owned by the
 * caller). stats (host, may be NULL) receives sums of the state f_in; with stats the call
 * synchronises, without it is asynchronous. One kernel launch (timed when timing is on).
 * Errors: KCF_EINVAL for NULL arguments, f_in == f_out, an unknown model, nu <= 0, c_nu < 0 or
 * n < 3; KCF_ENOMEM when the statistics records cannot be allocated. */
int kcf_lbm_step(kcf_ctx *ctx, const kcf_grid *grid, const kcf_lbm_params *params,
                 const float *f_in, float *f_out, kcf_lbm_stats *stats);

/* E_k, enstrophy and <rho> of the unfiltered input (synchronises). */
int kcf_input_stats(kcf_ctx *ctx, const kcf_grid *grid, const float *rho, const float *u,
                    kcf_input_summary *out);

/* FP64 sums over the GPU of arbitrary float32 device arrays, for checks of the reduction:
 * out[0] = sum a, out[1] = sum a^2, out[2] = sum a*b (b may be NULL: then out[2] = 0). */
int kcf_reduce_check(kcf_ctx *ctx, const float *a, const float *b, int64_t n, double *out);

/* ---- learned closure ------------------------------------------------------------------
 * A small MLP, 14 inputs -> 64 -> 64 -> 64 -> 6 outputs, GELU (tanh form) after the hidden
 * layers, maps the filtered velocity gradient to tau. The paper has no learned closure; this
 * is the interface of the learned part of the library:
 *   inputs  (14): g = Delta * G (G_ij = d_j ut_i, central differences, row-major) and the five
 *                 invariants tr(s^2), tr(r^2), tr(s^3), tr(s r^2), tr(s^2 r^2) of g, s and r being
 *                 its symmetric and antisymmetric parts;
 *   targets (6) : tau_c / rho_bar, c = xx xy xz yy yz zz;
 *   both standardised with training-set means and standard deviations.
 * Matrix products run on BF16 MFMA with FP32 accumulation (inputs, weights, activations and
 * back-propagated deltas are rounded to BF16 at the products); biases, GELU, loss and Adam
 * stay in FP32. Parameters: a float32 vector of 9670 values packed W1 (64x14), b1, W2 (64x64),
 * b2, W3 (64x64), b3, W4 (6x64), b4, each W row-major (out, in).
 * Normalisation block (68 floats): x_mean[14], x_std[14], y_mean[6], y_std[6], x_lo[14],
 * x_hi[14]; x_lo/x_hi bound the standardised inputs seen in training (the envelope). */
/* The context must outlive every network created on it. */
int kcf_mlp_create(kcf_ctx *ctx, kcf_mlp **out);  /* zero parameters, identity normalisation */
void kcf_mlp_destroy(kcf_mlp *mlp);
int kcf_mlp_set_params(kcf_mlp *mlp, const float *params_host);  /* also resets Adam state */
int kcf_mlp_get_params(kcf_mlp *mlp, float *params_host);
/* 68 floats, see above; KCF_EINVAL unless every std is finite and > 0 and every mean finite
 * (the envelope bounds may be infinite). */
int kcf_mlp_set_norm(kcf_mlp *mlp, const float *norm_host);
int kcf_mlp_get_norm(kcf_mlp *mlp, float *norm_host);
int kcf_mlp_step_count(kcf_mlp *mlp, int64_t *step);

/* Network inputs x_out (N rows of 14, device) and, when tau and y_out are given, targets
 * y_out (N rows of 6) of every grid point, from filtered fields of width delta. */
int kcf_mlp_features(kcf_ctx *ctx, const kcf_grid *grid, const float *rho_bar, const float *ut,
                     const float *tau, double delta, float *x_out, float *y_out);
/* FP64 column sums, sums of squares, minima and maxima of an n x ncol row-major device matrix
 * (host outputs; synchronises). ncol <= 32. */
int kcf_mlp_column_stats(kcf_ctx *ctx, const float *X, int64_t n, int ncol, double *sum,
                         double *sumsq, double *mn, double *mx);
/* Sets the normalisation from a training set (population standard deviations; envelope =
 * standardised per-column minima and maxima). */
int kcf_mlp_fit_norm(kcf_mlp *mlp, const float *x, const float *y, int64_t n);

/* One Adam step (lr, beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected) on the minibatch
 * rows idx[0..batch) of the dataset (x: n x 14, y: n x 6, raw, device; idx: device int32,
 * NULL = rows 0..batch-1). Indices must lie in [0, n); the kernel clamps them to that range.
 * batch: multiple of 32. loss_dev (device float, may be NULL) receives the batch MSE before
 * the update. Asynchronous. */
int kcf_mlp_train_step(kcf_mlp *mlp, const float *x, const float *y, int64_t n,
                       const int32_t *idx, int batch, float lr, float *loss_dev);
/* Loss and gradient of the current parameters on a minibatch (host outputs; synchronises). */
int kcf_mlp_grads(kcf_mlp *mlp, const float *x, const float *y, int64_t n, const int32_t *idx,
                  int batch, float *grads_host, double *loss_host);
/* Standardised network outputs (n rows of 6, device) for raw input rows x (n x 14). */
int kcf_mlp_predict(kcf_mlp *mlp, const float *x, int64_t n, float *y_std);
/* Learned tau (6N, symmetric-tensor blocks) over a field from rho_bar (N) and ut (3N) of
 * filter width delta. Points whose standardised inputs leave the envelope, or are not finite,
 * take the gradient model rho_bar * m2 * G G^T instead. mask (device, ceil(N/16) uint16
 * words, bit p of word t = point 16 t + p, may be NULL) marks those points; n_fallback (host,
 * may be NULL) counts them: when it is given the call synchronises the stream, with NULL the
 * call is asynchronous. */
int kcf_mlp_infer_field(kcf_mlp *mlp, const kcf_grid *grid, const float *rho_bar,
                        const float *ut, double delta, double m2, float *tau, uint16_t *mask,
                        int64_t *n_fallback);
/* Checkpoint of parameters, Adam moments, step count and normalisation, with a checksum.
 * Errors: KCF_EIO for unreadable, truncated, oversized or corrupted files (the network is
 * then unchanged), KCF_EINVAL for a checkpoint whose normalisation kcf_mlp_set_norm rejects. */
int kcf_mlp_save(kcf_mlp *mlp, const char *path);
int kcf_mlp_load(kcf_mlp *mlp, const char *path);

/* ---- measurement aid ----------------------------------------------------------------- */
/* Plain streaming kernel: out block j (n floats) = in block (j mod nin) times (j + 1), for
 * nin <= 8 input and nout <= 64 output blocks of n floats (device, caller-owned). It moves the
 * bytes of a call of the filtering path (4 fields in; 10 per width out) with no other work, so
 * its time is the practical HBM floor of such a call on the device. Asynchronous, timed like
 * the filter launches. Not part of the method. Errors: KCF_EINVAL for NULL or out-of-range
 * arguments. */
int kcf_stream_probe(kcf_ctx *ctx, const float *in, int nin, float *out, int nout, int64_t n);

#ifdef __cplusplus
}
#endif
#endif /* KCF_H */
