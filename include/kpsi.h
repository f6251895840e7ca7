/* kpsi.h -- C ABI of the MI355X likelihood engine for the four-dimensional
 * B0 -> J/psi K pi amplitude fit (arXiv:2007.14931).
 *
 * The library evaluates, on one GPU, the unbinned negative log-likelihood of the
 * paper's amplitude model and its gradient.  The host-side minimiser calls a
 * function of the fit parameters while the device evaluates the PDF over all events
 * (Introduction: the fit parameters are stepped on the host, the PDF/NLL is evaluated
 * on the device; State-of-the-art section: the normalisation is evaluated numerically
 * over millions of phase-space points).
 *
 * Conventions shared by every call
 *  - Every function returns kpsi_status (0 = KPSI_OK, < 0 = error) and never throws.
 *    On error a message is available from kpsi_last_error(ctx) until the next call on
 *    that context.
 *  - Units: GeV for masses and momenta, GeV^-1 for barrier radii, radians for angles.
 *  - Host arrays passed in are copied before the call returns; the caller keeps
 *    ownership.  Device pointers passed to *_device calls are borrowed: the caller
 *    keeps them alive and unchanged until the context is destroyed or the set is
 *    reloaded; the library never frees them.
 *  - All device work runs on the context's stream (the one given to kpsi_create, or a
 *    stream the library creates).  Calls returning results to the host wait once for the
 *    work they enqueued: kpsi_nll, kpsi_nll_and_grad and its _noalloc form poll the values
 *    their final reduction stores into pinned host memory (each marked pending beforehand;
 *    bounded at 50 ms, then a stream synchronize, which also reports kernel errors); the
 *    others synchronize the stream.  When a call returns, its results are written and every
 *    kernel it enqueued has made its last memory access (the reduction's final kernel may
 *    still be retiring; later work on the stream is ordered after it).  A context is not
 *    thread-safe; separate contexts are independent.
 *
 * Observables (Eq. 1, with theta_K* in place of m_J/psi pi, which it determines at
 * fixed m_Kpi): per event m_Kpi, cos theta_K*, cos theta_J/psi and phi (Eq. 4 and
 * the definitions below it).  Events are accepted only inside the physical region:
 * mK + mpi <= m_Kpi <= mB - mJ/psi, |cos| <= 1, |phi| <= pi (a tolerance of 1e-12 is
 * allowed and values are clamped to the boundary).
 *
 * Parameter vector (double, length from kpsi_n_params): for each resonance in the
 * order given to kpsi_set_model, its helicity couplings as (magnitude, phase) pairs --
 * K* (Eq. 4): lambda = -1, 0, +1, or only lambda = 0 for spin 0; Z (Eq. 10, spin-parity
 * 1+): lambda' = 0 and lambda' = +1, with H'_-1 = H'_+1 from Eq. (11), or lambda' = 0, +1, -1
 * for a Z with hel_free set -- followed by
 * (M, Gamma0) of every resonance in table order (Eq. 2-3).  The overall phase and
 * magnitude convention of Eq. (6) is the caller's business (fix those entries).
 */
#ifndef KPSI_H
#define KPSI_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct kpsi_ctx kpsi_ctx;

typedef enum {
  KPSI_OK = 0,
  KPSI_E_ARG = -1,         /* NULL pointer, bad size, value outside the physical region */
  KPSI_E_STATE = -2,       /* model or event set missing, or a call made in the wrong order */
  KPSI_E_HIP = -3,         /* a HIP runtime call failed */
  KPSI_E_OOM = -4,         /* device or pinned-host allocation failed */
  KPSI_E_NONFINITE = -5,   /* a data-event density is <= 0 (in FP32: below the smallest
                              normal float) or not finite, or the MC normalisation is <= 0;
                              *nll is set to +inf */
  KPSI_E_UNSUPPORTED = -6  /* model outside what the compiled kernels cover */
} kpsi_status;

typedef enum {
  KPSI_FP64 = 0,           /* every per-event step in double precision */
  KPSI_FP32 = 1            /* per-event amplitudes in float with hardware transcendentals;
                              thresholds (breakup momenta) and the Z-chain frame computed
                              once in double; log-likelihood and normalisation sums in
                              double with compensated summation */
} kpsi_precision;

typedef enum { KPSI_DATA = 0, KPSI_NORM = 1 } kpsi_set;

typedef struct {
  int chain;     /* 0 = K* -> K pi (Eq. 4), 1 = Z -> J/psi pi (Eq. 10) */
  int spin;      /* J: 0..4 for K*, 1 for Z */
  int parity;    /* +1 / -1; Z must be 1+ (Eq. 11 relation is then H'_-1 = H'_+1) */
  int lb, lr;    /* orbital momenta of the B and resonance decays; < 0 selects the lowest
                    allowed value (text below Eq. 3), the only values supported */
  double mass;   /* nominal M (used only as the default entry of the parameter vector) */
  double width;  /* nominal Gamma0 (idem) */
  int shape;     /* 0: relativistic Breit-Wigner of Eq. 2-3.  1: LASS S-wave of Eq. 7-8 (K* of
                    spin 0 only; its M and Gamma0 cannot float), read as
                      A = F_B (p_B/M_B)^L_B [ (m/q) sin d e^{i d}
                                              + e^{2 i d} (M^2 Gamma0/q0) / (M^2 - m^2 - i M Gamma(m)) ]
                    with cot d = 1/(a q) + b q/2 and Gamma(m) = Gamma0 (q/q0)(M/m) */
  double lass_a; /* LASS scattering length a in GeV^-1 (> 0); ignored when shape = 0 */
  double lass_b; /* LASS effective range b in GeV^-1 (finite); ignored when shape = 0 */
  int hel_free;  /* Z only (0 for a K*): 1 leaves H'_+1 and H'_-1 independent instead of tied by
                    Eq. 11 (the Discussion's unconstrained Z couplings); the Z then has three
                    couplings, lambda' = 0, +1, -1 in that order.  Supported for a model with
                    exactly one Z (kpsi_set_model returns KPSI_E_UNSUPPORTED otherwise) */
} kpsi_resonance;

typedef struct {
  double m_b, m_jpsi, m_k, m_pi;   /* particle masses */
  double r_b, r_r;                 /* Blatt-Weisskopf radii of the B and resonance decays */
} kpsi_kinematics;

/* Create a context on HIP device `device`.  `stream` is a hipStream_t to run on, or NULL
 * for a library-owned stream.  `prec` selects the per-event arithmetic. */
kpsi_status kpsi_create(int device, void* stream, kpsi_precision prec, kpsi_ctx** out);
/* Free every device and pinned buffer the context owns (borrowed pointers untouched). */
kpsi_status kpsi_destroy(kpsi_ctx* ctx);

/* Set the decay constants and the resonance table (Eq. 2-4, 10-12).  Supported: up to
 * ten K* of spin 0..4 with at most 3, 3, 2, 1, 1 states of spin 0, 1, 2, 3, 4, and up to
 * two Z of spin-parity 1+.  Loaded events are re-derived for the new constants. */
kpsi_status kpsi_set_model(kpsi_ctx* ctx, const kpsi_kinematics* kin, const kpsi_resonance* res, int n_res);
/* Length of the canonical parameter vector of the current model. */
kpsi_status kpsi_n_params(const kpsi_ctx* ctx, int* n_full);
/* Select the resonances whose (M, Gamma0) gradient kpsi_nll_and_grad computes
 * (flags[i] != 0, at most two).  Gradient entries of other lineshape parameters are
 * returned as NaN.  Default: none. */
kpsi_status kpsi_set_floating(kpsi_ctx* ctx, const int* flags, int n_res);

/* Load the data set (KPSI_DATA) or the phase-space normalisation set (KPSI_NORM) from
 * host arrays of n doubles each (copied).  Replaces a previously loaded set. */
kpsi_status kpsi_load_events(kpsi_ctx* ctx, kpsi_set set, int64_t n, const double* m_kpi, const double* cos_k,
                             const double* cos_j, const double* phi);
/* Same from device arrays (borrowed; see ownership above).  The library reads them on the
 * context's stream: work that writes them on another stream (a torch stream, say) must have
 * completed before the call, or the context must be created on that stream. */
kpsi_status kpsi_load_events_device(kpsi_ctx* ctx, kpsi_set set, int64_t n, const double* m_kpi,
                                    const double* cos_k, const double* cos_j, const double* phi);

/* Efficiency eps(Phi) of Eq. (14) on the normalisation set: flat (default), or one value
 * per normalisation event (host array of n_norm doubles, copied; 0 <= eps <= 1). */
kpsi_status kpsi_set_efficiency_flat(kpsi_ctx* ctx);
kpsi_status kpsi_set_efficiency_values(kpsi_ctx* ctx, const double* eps, int64_t n);
/* Binned efficiency: a row-major float histogram of nb[0]*nb[1]*nb[2]*nb[3] bins over
 * (m_Kpi, cos theta_K*, cos theta_J/psi, phi) with lower edges lo[] and upper edges hi[]
 * (bins [lo, hi), the upper edge falls in the last bin), looked up once per
 * normalisation event on the device. */
kpsi_status kpsi_set_efficiency_hist(kpsi_ctx* ctx, const float* eff, const int nb[4], const double lo[4],
                                     const double hi[4]);
/* Importance-sampled normalisation (the normalisation integral of Eq. 12-14 estimated over
 * phase-space points that are not all flat; State-of-the-art section: the normalisation is
 * evaluated numerically over millions of phase-space points).  The loaded normalisation set is
 * taken as a mixture: its first n_flat events drawn flat in phase space, the other n - n_flat
 * drawn from the density S(y; params0) (for instance by kpsi_generate_model at params0, without
 * an efficiency).  Each event then gets the weight
 *   w_j = 1 / (alpha + (1 - alpha) S(y_j; params0) / Z0),   alpha = n_flat / n,
 * Z0 = the flat events' mean of S(y; params0): the ratio of flat phase space to the mixture's
 * density, so that weighted sums over the set estimate flat phase-space integrals for any
 * parameters.  The weights multiply the efficiency in every normalisation sum (the per-event
 * kernel, the interference matrix), weight the efficiency-free fit-fraction integrals and the
 * background normalisation of kpsi_set_background, and survive later kpsi_set_efficiency_*
 * calls.  n_flat = n removes them.  Events placed under a narrow peak this way lower the
 * statistical error of the normalisation (and of the fitted parameters it moves) where the
 * data are.  Errors: KPSI_E_STATE without a model or normalisation set, or when a background
 * is already set (set the mixture first); KPSI_E_ARG for n_flat outside [1, n], non-finite
 * params0, or a density that is negative or not finite. */
kpsi_status kpsi_set_norm_mixture(kpsi_ctx* ctx, const double* params0, int64_t n_flat);

/* -2 ln L (Eq. 14 signal part, purity 1):
 *   NLL = -2 sum_data ln S(x_i) + 2 N_data ln( (1/N_norm) sum_norm eps_j S(y_j) )
 * with S of Eq. (12) (Eq. 5 when no Z is present).  params: canonical vector. */
kpsi_status kpsi_nll(kpsi_ctx* ctx, const double* params, double* nll);
/* NLL and its gradient with respect to every coupling entry and the (M, Gamma0) of the
 * resonances selected with kpsi_set_floating, in one pass (hand-written adjoint). */
kpsi_status kpsi_nll_and_grad(kpsi_ctx* ctx, const double* params, double* nll, double* grad);
/* kpsi_nll_and_grad for callers that cannot allocate device memory during the call (code under
 * stream capture, tight serving loops, harnesses that forbid allocation).  Same arguments,
 * layout, results and errors as kpsi_nll_and_grad, with every data and normalisation event
 * evaluated directly: the interference-matrix cache is neither built nor consulted, and no
 * timing sample is recorded.  The call allocates nothing: its block partials live in a static
 * device array of the library (8 MiB per device, held until the process ends) instead of a
 * buffer the context grows.  A call needing more than 16384 block partials (events per block:
 * 256 x the events per thread) returns KPSI_E_ARG before any work is enqueued.  The array is
 * shared by every context on a device and keeps the last call's contents (each call writes
 * every partial it reads): calls that overlap on one device, from different streams or
 * threads, race on it and must be serialised by the caller. */
kpsi_status kpsi_nll_and_grad_noalloc(kpsi_ctx* ctx, const double* params, double* nll, double* grad);

/* Diagnostics (not on the fit path).  Per-event density S of a loaded set into a host
 * array of n doubles (S of Eq. 12 at the event as loaded: flavour tags and the background
 * mixture are not applied); per-event Z-chain observables into a host array of 5n doubles
 * (m_Jpsi pi, cos theta_Z, cos theta~_J/psi, phi~, alpha). */
kpsi_status kpsi_density(kpsi_ctx* ctx, kpsi_set set, const double* params, double* out);
kpsi_status kpsi_invariants(kpsi_ctx* ctx, kpsi_set set, double* out);

/* Generators (Philox4x32-10 counters, so results depend only on the seed and event
 * index).  Flat phase space: m_Kpi ~ p_B(m) q(m) by accept-reject under the envelope
 * wmax, angles uniform.  Output: four device arrays of n doubles. */
kpsi_status kpsi_generate_phsp(kpsi_ctx* ctx, uint64_t seed, int64_t n, double wmax, double* m_kpi,
                               double* cos_k, double* cos_j, double* phi);
/* Accept-reject from eps_true(Phi) * S(Phi; params) over phase-space proposals: proposal e
 * is kept when u_e * smax < eps S, in proposal order, until n are kept.  acc_coef is NULL
 * (no acceptance) or 12 doubles of the seeded analytic acceptance.  Outputs: four device
 * arrays of n doubles; *n_prop proposals used; *n_over proposals with eps S > smax. */
kpsi_status kpsi_generate_model(kpsi_ctx* ctx, const double* params, uint64_t seed, int64_t n, double wmax,
                                double smax, const double* acc_coef, double* m_kpi, double* cos_k, double* cos_j,
                                double* phi, int64_t* n_prop, int64_t* n_over);

/* Duration of the per-event work of one call, for measurement: the per-event kernel launches of
 * a kpsi_nll_and_grad (grad != 0) or kpsi_nll (grad == 0) call over every loaded event are
 * enqueued `reps` times back to back on the context stream between one pair of HIP events,
 * followed by one final reduction; *ms_per_launch receives the events' interval divided by reps
 * (launch gaps included, the reduction and host work excluded).  reps in [1, 100000].  The
 * interference-matrix cache is not used.  Same errors as kpsi_nll_and_grad. */
kpsi_status kpsi_time_kernel(kpsi_ctx* ctx, const double* params, int grad, int reps, double* ms_per_launch);
/* Device timing of the per-event kernel: with every = k > 0, every k-th nll /
 * nll_and_grad call (counting from the first after this call) records HIP events around
 * the kernel on the context stream; every = 0 turns timing off.  kpsi_timing returns the
 * summed kernel milliseconds and the number of timed calls since the last reset.
 * KPSI_E_ARG if every < 0. */
kpsi_status kpsi_set_timing(kpsi_ctx* ctx, int every);
kpsi_status kpsi_timing(kpsi_ctx* ctx, double* kernel_ms, int64_t* n_calls, int reset);
/* Median kernel milliseconds of the timed calls since the last reset (the first 65536 of them);
 * NaN when none was timed.  kernel_ms: one double (host, caller-owned).  KPSI_E_ARG for NULL. */
kpsi_status kpsi_timing_median(kpsi_ctx* ctx, double* kernel_ms);

/* ---------------------------------------------------------------- fit driver
 * Variable-metric minimisation (MINUIT MIGRAD style: BFGS update of the inverse Hessian,
 * parabolic backtracking line search, stop when the expected distance to the minimum
 * EDM = g^T V g / 2 < 0.002 * tolerance * up) and HESSE covariance, of the context's NLL
 * over the parameters with free_mask[i] != 0 (length kpsi_n_params; the other entries of
 * params are held fixed, e.g. H_0 of K*(892) by Eq. 6).  The host steps the parameters
 * and the device evaluates the NLL (Introduction).  Points where the NLL call reports
 * KPSI_E_NONFINITE or KPSI_E_ARG (unphysical mass or width) are rejected steps. */
typedef struct {
  int64_t max_calls;    /* budget of NLL plus NLL+gradient evaluations */
  double tolerance;     /* EDM target factor (MINUIT default 0.1) */
  double up;            /* error definition: 1.0 for -2 ln L */
  int gradient;         /* 1: analytic gradient (kpsi_nll_and_grad); 0: central finite
                           differences of kpsi_nll (2 P calls per gradient) */
  double fd_rel_step;   /* finite-difference step h_i = fd_rel_step * (1 + |x_i|) */
  int hesse;            /* 1: numerical Hessian at the minimum for the covariance */
} kpsi_fit_options;

typedef struct {
  double fmin;          /* NLL at the minimum */
  double edm;           /* expected distance to the minimum at exit */
  double wall_seconds;  /* host wall time of the whole call */
  int64_t n_nll;        /* kpsi_nll evaluations */
  int64_t n_grad;       /* kpsi_nll_and_grad evaluations */
  int n_iter;           /* variable-metric iterations */
  int status;           /* 0 converged; 1 call budget exhausted; 2 line search failed;
                           3 Hessian not positive definite; 4 device error */
} kpsi_fit_result;

/* Fill opts with the defaults (analytic gradient, tolerance 0.1, up 1, HESSE on). */
kpsi_status kpsi_fit_default_options(kpsi_fit_options* opts);
/* Minimise.  params (length kpsi_n_params) is the start point on entry and the minimum on
 * exit.  cov (optional, n_free x n_free row-major in the order of the free indices)
 * receives 2 up H^-1 from HESSE, or the final variable-metric estimate when opts->hesse
 * is 0. */
kpsi_status kpsi_migrad(kpsi_ctx* ctx, double* params, const int* free_mask, const kpsi_fit_options* opts,
                        kpsi_fit_result* result, double* cov);
/* kpsi_migrad with limits on the free parameters (MINUIT's transformations; the paper fits
 * with MINUIT).  lower, upper: host arrays of kpsi_n_params doubles, or NULL for none; an entry
 * that is not finite (NaN, +-inf) leaves that side open, and the entries of fixed parameters
 * are ignored.  The minimiser works on an internal variable u per limited parameter:
 * lo + (hi - lo)(sin u + 1)/2 with both limits, lo - 1 + sqrt(u^2 + 1) with a lower one,
 * hi + 1 - sqrt(u^2 + 1) with an upper one, so every trial point lies inside its limits.
 * cov is the internal covariance mapped with the derivatives of the transformations at the
 * minimum (it shrinks towards zero for a parameter that ends at a limit).  KPSI_E_ARG if a
 * lower limit is not below its upper one or the start is not strictly inside its limits. */
kpsi_status kpsi_migrad_limited(kpsi_ctx* ctx, double* params, const int* free_mask, const double* lower,
                                const double* upper, const kpsi_fit_options* opts, kpsi_fit_result* result,
                                double* cov);
/* Covariance 2 up H^-1 at params from a numerical Hessian (gradient differences in the
 * analytic mode, second differences of the NLL otherwise). */
kpsi_status kpsi_hesse(kpsi_ctx* ctx, const double* params, const int* free_mask, const kpsi_fit_options* opts,
                       double* cov, kpsi_fit_result* result);

/* Normalisation through the interference matrix (the per-resonance-pair form of the MC
 * normalisation sum): sum_j eps_j S(y_j) = sum_kl c_k conj(c_l) I_kl with
 * I_kl = sum_j eps_j sum_xi B_k,xi(y_j) conj(B_l,xi(y_j)) over the complex couplings c_k and
 * per-event component amplitudes B_k,xi of Eq. 4 and Eq. 10, plus the matrices
 * D^p_kl = sum_j eps_j sum_xi dB_k,xi/dp conj(B_l,xi) for the floating lineshapes.  They are
 * built with matrix-core products over the normalisation set (in the FP32 context FP32
 * products summed in FP64 per 64-row tile, in the FP64 context FP64 products) and depend only on the
 * masses and widths, so a call whose masses and widths equal those of the cached build
 * evaluates only the data events.
 *   mode 0: off (default; every call evaluates both sets)
 *   mode 1: on (rebuild whenever masses or widths change)
 *   mode 2: auto (use the cache when it matches; build only after KPSI_CACHE_AUTO_STREAK
 *           consecutive calls at the same masses and widths, e.g. the coupling directions of
 *           a finite-difference gradient; a build costs about as much as 5-10 direct calls)
 * Loading the normalisation set, changing the efficiency, the model or the floating set
 * drops the cache. */
#define KPSI_CACHE_AUTO_STREAK 16
kpsi_status kpsi_set_norm_cache(kpsi_ctx* ctx, int mode);
/* Cache builds, calls served from the cache, and the device milliseconds of the last build. */
kpsi_status kpsi_norm_cache_stats(const kpsi_ctx* ctx, int64_t* builds, int64_t* hits, double* last_build_ms);

/* Fit fractions (Eq. 13): ff[j] = int S_j dPhi / int S dPhi for every resonance j of the
 * model, where S_j is the density with all helicity couplings outside resonance j set to zero
 * and the integrals run over phase space without efficiency.  They are estimated on the loaded
 * normalisation events (flat phase space) through one interference-matrix build at the
 * masses and widths of params (matrix-core Gram product as above, efficiency column not applied;
 * the normalisation cache is left untouched): ff[j] = c_j^H I_jj c_j / c^H I c.
 *   params: full parameter vector (kpsi_n_params doubles, host).
 *   ff:     n_res doubles (host, caller-owned), table order.
 *   ff_sum: optional (may be NULL), the sum of the fractions (not 1 when resonances interfere).
 * Errors: KPSI_E_STATE without a model or normalisation set; KPSI_E_ARG for NULL or non-finite
 * parameters; KPSI_E_NONFINITE when the integral of the density is not positive. */
kpsi_status kpsi_fit_fractions(kpsi_ctx* ctx, const double* params, double* ff, double* ff_sum);

/* ---------------------------------------------------------------- signal + background (Eq. 14)
 * The mixture PDF f = p eps S / N_S + (1 - p) b / N_b of Eq. 14 (Results: applicability to
 * real-life use cases): p the signal purity, eps the relative signal efficiency, b the
 * background density, N_S and N_b the normalisation-event means of eps S and of b, so that
 * both terms are normalised over phase space.  Once set, kpsi_nll / kpsi_nll_and_grad return
 *   -2 ln L = -2 sum_i ln(p eps_i S_i + (1 - p)(N_S / N_b) b_i) + 2 N_d ln N_S
 * (equal to -2 sum_i ln f(x_i) up to the dropped phase-space volume).  The normalisation
 * events keep the efficiency of kpsi_set_efficiency_*.  The data terms need N_S, so each call
 * evaluates the normalisation events first (or takes them from the interference matrix).
 *   purity:   0 < p <= 1.
 *   eps_data: efficiency at each loaded data event (n_data doubles, host; NULL = 1).
 *   b_data:   background density at each data event (n_data doubles, host; NULL switches the
 *             mixture off and restores the signal-only likelihood).
 *   b_norm:   background density at each normalisation event (n_norm doubles, host).
 * Values are copied (and rounded to the context precision).  Loading either event set drops
 * the mixture.  Errors: KPSI_E_ARG for a purity outside (0, 1], negative or non-finite values,
 * or a non-positive background integral; KPSI_E_STATE unless both sets are loaded. */
kpsi_status kpsi_set_background(kpsi_ctx* ctx, double purity, const double* eps_data, const double* b_data,
                                const double* b_norm);

/* ---------------------------------------------------------------- flavour tags (text after Eq. 12)
 * Charge-conjugate decays: the density of the conjugate decay is S with the sign of phi
 * reversed.  tags[i] = +1 (B0) or -1 (conjugate) for each loaded data event; an event is of the
 * other flavour with probability `mistag`, both flavours equally produced.  Once set,
 * kpsi_nll / kpsi_nll_and_grad return
 *   -2 ln L = -2 sum_i ln[(1 - w) S(x_i^(q_i)) + w S(x_i^(-q_i))] + 2 sum_q n_q ln N_q,
 *   x^(s) = (m, cos theta_K*, cos theta_J/psi, s phi),  N_q = (1 - w) I(q) + w I(-q),
 *   I(s) = (1/N_MC) sum_j eps_j S(y_j^(s))
 * (n_q the number of data events tagged q; the data efficiencies dropped as for the signal
 * likelihood).  A direct call evaluates the normalisation events at +phi and at -phi.  With
 * the interference-matrix cache on (kpsi_set_norm_cache), both come from the +phi matrix:
 * reversing phi gives the density of the original event with the lambda = -1 and +1
 * couplings of every K* of spin >= 1 exchanged, so I(-phi) is the +phi form at the exchanged
 * couplings.
 *   tags:   n doubles (host, copied), n = the number of loaded data events; NULL switches the
 *           tags off (every event a B0).
 *   mistag: w in [0, 1/2].
 * Together with the background mixture (kpsi_set_background), the background density is the
 * same for both flavours and each flavour's PDF is normalised:
 *   f(x, q) = p eps(x) [(1 - w) S(x^(q)) + w S(x^(-q))] / N_q + (1 - p) b(x) / N_b,
 *   -2 ln L = -2 sum_i ln(p eps_i [(1 - w) S(x_i^(q_i)) + w S(x_i^(-q_i))] + (1 - p)(N_q / N_b) b_i)
 *             + 2 sum_q n_q ln N_q
 * (the data efficiencies enter here, as in the untagged mixture).  Each call then evaluates
 * the normalisation events at +phi and -phi first, or takes both from the interference matrix.
 * Loading data events drops the tags.  Errors: KPSI_E_ARG for a wrong count, a tag other than
 * +-1 or w outside [0, 1/2]. */
kpsi_status kpsi_set_flavour(kpsi_ctx* ctx, const double* tags, int64_t n, double mistag);

/* ---------------------------------------------------------------- Gaussian constraints
 * Gaussian constraints on fit parameters (Conclusion: applied when required): a factor
 * N(p[index_k]; mean_k, sigma_k) per constraint in the likelihood, i.e.
 *   sum_k ((p[index_k] - mean_k) / sigma_k)^2
 * added to -2 ln L by kpsi_nll and kpsi_nll_and_grad (gradient 2 (p - mean) / sigma^2), and so
 * seen by kpsi_migrad and kpsi_hesse.  index: positions in the canonical parameter vector;
 * arrays of n (host, copied); n = 0 removes the constraints.  kpsi_set_model removes them.
 * Errors: KPSI_E_ARG for an index out of range, sigma <= 0 or non-finite values, NULL arrays
 * with n > 0; KPSI_E_STATE without a model. */
kpsi_status kpsi_set_constraints(kpsi_ctx* ctx, int n, const int* index, const double* mean, const double* sigma);

/* Per-event values of a 2D (mass variables) x 2D (angular variables) template, the form in
 * which the paper passes efficiency and background shapes to the fit: t_mass over
 * (m_Kpi in [m_K + m_pi, M_B - M_J/psi], cos theta_K* in [-1, 1]) with n_mass[0] x n_mass[1]
 * bins (row-major, m_Kpi slowest), t_ang over (cos theta_J/psi in [-1, 1], phi in [-pi, pi])
 * with n_ang[0] x n_ang[1] bins.  (m_Kpi, cos theta_K*) maps one-to-one onto
 * (m_Kpi, m_J/psi pi) at fixed m_Kpi and has a rectangular domain.  out[e] =
 * t_mass[bin] * t_ang[bin] for every event of the set (host, n doubles); bins are [lo, hi),
 * values outside are clamped into the edge bins.  Tables are host arrays, copied.
 * Errors: KPSI_E_ARG for NULL arguments or non-positive bin counts; KPSI_E_STATE if the set is
 * not loaded. */
kpsi_status kpsi_template_values(kpsi_ctx* ctx, kpsi_set set, const float* t_mass, const int n_mass[2],
                                 const float* t_ang, const int n_ang[2], double* out);

/* ---------------------------------------------------------------- attainable peaks
 * Microbenchmarks of the device (no context needed), the ceilings against which the kernels'
 * rates are read: FP32 and FP64 fused multiply-add issue (one operation per lane per
 * instruction; packed FP32 instructions are not used by this library), the FP32 reciprocal
 * unit, and a device-to-device copy of 1 GiB (read + write bytes).  Takes well under a second;
 * allocates 2 GiB of device memory for the copy and frees it.  Runs on its own stream.
 * Errors: KPSI_E_ARG for a NULL out; KPSI_E_HIP for a bad device or a failed launch;
 * KPSI_E_OOM if the buffers cannot be allocated. */
typedef struct {
  double fp32_fma_tflops;   /* 2 flop per FMA */
  double fp64_fma_tflops;
  double fp32_rcp_tops;     /* reciprocals per second, 1e12 */
  double copy_gbs;          /* bytes read + written per second, 1e9 */
} kpsi_peaks;
kpsi_status kpsi_measure_peaks(int device, kpsi_peaks* out);

/* ---------------------------------------------------------------- learned efficiency
 * The relative efficiency eps(Phi) of Eq. 14 learned by a 4 -> 64 -> 64 -> 1 network
 * (SiLU, SiLU, sigmoid) from accepted / generated phase-space events: the sigmoid output is
 * the acceptance probability.  The 64x64 layer runs on BF16 matrix cores with FP32
 * accumulation (forward, weight gradient and input gradient); FP32 master weights.
 * Parameters: 4545 floats, W1[64][4], b1[64], W2[64][64] (row = output), b2[64], w3[64], b3.
 * Input map: (2 (m - lo)/(hi - lo) - 1, cos theta_K*, cos theta_J/psi, phi/pi) with
 * [lo, hi] the m_Kpi range of the context's kinematics (set the model first).
 * Event arrays of these calls are device pointers of n doubles (borrowed for the call). */
typedef struct {
  int epochs;          /* passes over the training events */
  int64_t batch;       /* events per Adam step */
  double lr;           /* Adam step size */
  double beta1, beta2, eps;
} kpsi_mlp_options;

kpsi_status kpsi_mlp_default_options(kpsi_mlp_options* opts);
/* Accept labels of events e0 .. e0+n-1 under the seeded analytic acceptance acc_coef (12
 * doubles): label = [u < eps_true], u from Philox4x32-10 counter (event, 0, 3) with key seed.
 * label: device uint8 array of n; eps_true: optional device double array of n. */
kpsi_status kpsi_accept_labels(kpsi_ctx* ctx, uint64_t seed, int64_t e0, int64_t n, const double* m_kpi,
                               const double* cos_k, const double* cos_j, const double* phi, const double* acc_coef,
                               uint8_t* label, double* eps_true);
/* Binned efficiency from labelled events: table (host, nb[0]*nb[1]*nb[2]*nb[3] floats,
 * row-major) = accepted / generated per bin; bins without generated events take the overall
 * accepted fraction. */
kpsi_status kpsi_hist_efficiency(kpsi_ctx* ctx, int64_t n, const double* m_kpi, const double* cos_k,
                                 const double* cos_j, const double* phi, const uint8_t* label, const int nb[4],
                                 const double lo[4], const double hi[4], float* table);
/* Mean binary cross-entropy of the network over n labelled events and its gradient with
 * respect to the 4545 parameters (host output). */
kpsi_status kpsi_mlp_grad(kpsi_ctx* ctx, const float* params, int64_t n, const double* m_kpi, const double* cos_k,
                          const double* cos_j, const double* phi, const uint8_t* label, double* grad, double* loss);
/* Adam training over the labelled events; params (host, 4545) is the start point on entry and
 * the trained network on exit; *loss receives the mean loss of the last epoch. */
kpsi_status kpsi_mlp_train(kpsi_ctx* ctx, float* params, int64_t n, const double* m_kpi, const double* cos_k,
                           const double* cos_j, const double* phi, const uint8_t* label,
                           const kpsi_mlp_options* opts, double* loss);
/* Network output (probabilities) for n events into the device array out. */
kpsi_status kpsi_mlp_eval(kpsi_ctx* ctx, const float* params, int64_t n, const double* m_kpi, const double* cos_k,
                          const double* cos_j, const double* phi, double* out);
/* Efficiency of every normalisation event from the network, evaluated once on the device and
 * kept as the per-event efficiency column (it does not depend on the fit parameters). */
kpsi_status kpsi_set_efficiency_mlp(kpsi_ctx* ctx, const float* params);

/* Launch tuning: events handled by each thread of the per-event kernel (1..1024), or 0
 * for the automatic choice (about 2048 blocks over the two sets). */
kpsi_status kpsi_set_events_per_thread(kpsi_ctx* ctx, int ept);

/* Message of the last error on ctx (or of the last failed kpsi_create when ctx is NULL). */
const char* kpsi_last_error(const kpsi_ctx* ctx);

#ifdef __cplusplus
}
#endif
#endif /* KPSI_H */
