/* heget: per-event tree-level Standard Model helicity amplitudes on gfx950.
 *
 * C ABI of the library libheget.so.  The calls follow the paper's statement of
 * the problem (Sec. 2): for a partonic process a b -> 1 ... n, the squared
 * matrix element summed over helicities and colours,
 *     F = sum_lambda sum_c |M_lambda^c|^2,   M = sum over Feynman diagrams,
 * evaluated per phase-space point, and the cross section
 *     sigma = 1/(2 s) * 1/4 * 1/(n_a n_b) * 1/S * integral F dPhi_n
 * (the paper's LO partonic cross section and invariant phase space, Sec. 2;
 * S is the identical-particle symmetry factor).  A process is described by a
 * process IR: external legs, SM inputs, the list of HEGET-style vertex and
 * propagator calls (Sec. 4, Tables of external-line and vertex functions), the
 * decomposition of the amplitudes into colour flows and the colour matrix
 * (Sec. 5.4).
 *
 * Memory: every pointer argument of heget_eval / heget_integrate that is
 * documented as "device" must point to device memory of the current HIP device
 * and stay valid until the work enqueued on `stream` completes; the caller owns
 * it.  The IR passed to heget_process_create is host memory, read during the
 * call only (the library copies what it keeps).  A process handle owns its
 * device-resident tables and releases them in heget_process_destroy.
 *
 * Errors: every call returns a heget_status; no call aborts or throws.  On a
 * non-OK status, heget_last_error() returns a thread-local message.
 * Threading: a handle is immutable after creation; concurrent heget_eval calls
 * on one handle are allowed on different streams.
 */
#ifndef HEGET_H
#define HEGET_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  HEGET_OK = 0,
  HEGET_E_INVALID = -1,      /* bad argument (null pointer, n < 0, size mismatch) */
  HEGET_E_IR = -2,           /* the IR is malformed (slot, arity, kind or symmetry error) */
  HEGET_E_OOM = -3,          /* device allocation failed */
  HEGET_E_HIP = -4,          /* a HIP runtime call failed */
  HEGET_E_UNSUPPORTED = -5   /* no compiled kernel for this IR structure */
} heget_status;

typedef enum { HEGET_FP64 = 0, HEGET_MIXED = 1 } heget_precision;

/* leg kinds and particle ids (masses / widths) */
enum { HEGET_LEG_F = 0, HEGET_LEG_V = 1, HEGET_LEG_S = 2 };
enum { HEGET_P_ZERO = 0, HEGET_P_W = 1, HEGET_P_Z = 2, HEGET_P_TOP = 3, HEGET_P_H = 4, HEGET_N_PARTICLES = 5 };

/* call opcodes: HEGET function equivalents (paper Sec. 4, App. C) */
enum {
  HEGET_OP_IOV = 0, HEGET_OP_FVI, HEGET_OP_FVO, HEGET_OP_JIO,   /* FFV */
  HEGET_OP_IOS, HEGET_OP_FSI, HEGET_OP_FSO, HEGET_OP_HIO,       /* FFS */
  HEGET_OP_VVV, HEGET_OP_JVV,                                   /* VVV */
  HEGET_OP_GGGG, HEGET_OP_JGGG, HEGET_OP_WWWW, HEGET_OP_JWWW,   /* VVVV */
  HEGET_OP_VVS, HEGET_OP_JVS, HEGET_OP_HVV,                     /* VVS */
  HEGET_OP_VVSS, HEGET_OP_JVSS, HEGET_OP_HVVS,                  /* VVSS */
  HEGET_OP_SSS, HEGET_OP_HSS, HEGET_OP_SSSS, HEGET_OP_HSSS,     /* SSS, SSSS */
  HEGET_OP_VADD, HEGET_OP_VSUB,  /* in0 +- in1 for two currents of one momentum (coupling -1) */
  HEGET_N_OPS
};

/* coupling kinds; values are derived by the library from heget_sm */
enum {
  HEGET_CPL_GAMMA_FF = 0, /* photon-fermion, charge Q:      gc0 = gc1 = -e Q */
  HEGET_CPL_Z_FF,         /* Z-fermion, Q and T3:           gc0 = -g_Z (T3 - Q s_W^2), gc1 = g_Z Q s_W^2 */
  HEGET_CPL_W_FF,         /* W-fermion pair (CKM = 1):      gc0 = -g_W / sqrt2, gc1 = 0 */
  HEGET_CPL_G_QQ,         /* quark-gluon, colour -T^a:      gc0 = gc1 = g_s */
  HEGET_CPL_GGG,          /* triple gluon, colour i f^abc:  g_s */
  HEGET_CPL_GGGG,         /* four gluon, colour f f:        g_s^2 */
  HEGET_CPL_WWZ,          /* g_W cos theta_W */
  HEGET_CPL_WWA,          /* e */
  HEGET_CPL_WWH,          /* g_W m_W (complex mass in the complex-mass scheme) */
  HEGET_CPL_ZZH,          /* g_Z m_Z */
  HEGET_CPL_WWHH,         /* g_W^2 / 2 */
  HEGET_CPL_ZZHH,         /* g_Z^2 / 2 */
  HEGET_CPL_HHH,          /* -3 m_H^2 / v */
  HEGET_CPL_HHHH,         /* -3 m_H^2 / v^2 */
  HEGET_CPL_HBB,          /* gc0 = gc1 = -m_b / v  (Yukawa mass mb_yuk) */
  HEGET_CPL_WWWW,         /* -g_W^2  (W-W+W-W+) */
  HEGET_CPL_WWZZ,         /* g_W^2 cos^2 theta_W  (W-ZW+Z) */
  HEGET_N_CPL
};

typedef struct {
  double alpha;         /* QED coupling */
  double sw2;           /* sin^2 theta_W */
  double mz, wz;        /* Z mass, width (GeV) */
  double mw, ww;        /* W mass, width; ignored when complex_mass != 0 */
  double mt, wt;        /* top mass, width */
  double mh, wh;        /* Higgs mass, width */
  double alpha_s;       /* strong coupling */
  double mb_yuk;        /* b mass entering the Yukawa coupling only */
  int32_t complex_mass; /* 1: m_V^2 -> m_V^2 - i m_V Gamma_V in propagators and couplings,
                           with mu_W^2 = c_W^2 mu_Z^2 (paper, complex-mass discussion of Sec. 6) */
} heget_sm;

typedef struct {
  int32_t kind;      /* HEGET_LEG_F / _V / _S */
  int32_t incoming;  /* 1 = initial state, 0 = final state */
  int32_t flow;      /* fermions: +1 particle, -1 antiparticle (ignored otherwise) */
  int32_t particle;  /* HEGET_P_* : mass and width of the external line */
  int32_t colour;    /* 1, 3 or 8 */
} heget_leg;

typedef struct {
  int32_t kind;      /* HEGET_CPL_* */
  int32_t particle;  /* reserved (0) */
  double charge;     /* Q for photon / Z couplings */
  double t3;         /* T3 for Z couplings */
} heget_coupling;

typedef struct {
  int32_t op;        /* HEGET_OP_* */
  int32_t in[4];     /* input slots in argument order; -1 for unused */
  int32_t out;       /* output slot (currents) or amplitude index (amplitude ops) */
  int32_t coupling;  /* index into heget_process_ir.couplings */
  int32_t prop;      /* HEGET_P_* of the propagator of a current (0 for amplitudes) */
} heget_call;

/* Resonance phase space (the paper's Appendix A, Eqs. for the Breit-Wigner
 * parametrisation, at a fixed collision energy): the collision system and every
 * resonance decay into two daughters (isotropic in the parent's rest frame);
 * dPhi_n = dPhi_2(collision) prod_k ds_k / (2 pi) dPhi_2(resonance k at s_k).
 * A resonance's s_k follows the Breit-Wigner mapping s = m^2 + m Gamma tan(theta),
 * theta uniform over |s - m^2| / (m Gamma) < min(ps_window, m / Gamma) intersected
 * with the kinematic range, or a flat distribution over the kinematic range.
 * A final particle has the mass of its leg's particle (HEGET_P_ZERO: massless);
 * a node's minimal mass is the sum of the final masses below it, and the ranges
 * are [min_first^2, (M - min_second)^2] for the first daughter of a node of
 * mass M, [min_second^2, (M - m_first)^2] for the second. */
enum { HEGET_PS_FLAT = 0, HEGET_PS_BREIT_WIGNER = 1 };
typedef struct {
  int32_t particle;     /* HEGET_P_* giving the resonance's mass and width (node 0, the collision: ignored) */
  int32_t mapping;      /* HEGET_PS_FLAT or HEGET_PS_BREIT_WIGNER (node 0: ignored) */
  int32_t daughter[2];  /* final leg index (2 .. n_legs-1), or -1 - k for node k > this node */
} heget_ps_node;

/* Slots 0 .. n_legs-1 hold the external wavefunctions; every current writes a
 * new slot >= n_legs that is read only by later calls. */
typedef struct {
  int32_t n_legs;
  const heget_leg* legs;              /* [n_legs]; legs 0 and 1 are the incoming partons */
  heget_sm sm;
  int32_t n_couplings;
  const heget_coupling* couplings;
  int32_t n_calls;
  const heget_call* calls;
  int32_t n_amps;
  int32_t n_flows;
  const double* jamp;                 /* [rows][n_amps][2]: J_f = sum_a jamp[f][a] * amp_a; rows =
                                         n_flows, or n_orderings for an ordering template */
  const double* colour_num;           /* [n_flows][n_flows] symmetric numerators */
  double colour_den;                  /* colour matrix = colour_num / colour_den */
  int32_t n_hel;
  const int8_t* helicities;           /* [n_hel][n_legs]: -1, 0, +1 (4 = gauge vector k/k^0) */
  int32_t n_a_n_b;                    /* initial-state colour degrees of freedom n_a n_b */
  int32_t symmetry;                   /* identical-particle factor S */
  int32_t cut_enabled;                /* every final leg pT > cut_pt and every pair Delta R > cut_dr */
  double cut_pt, cut_dr;
  /* Ordering table (colour-ordered processes), or n_orderings = 0.  When set,
   * the calls form a template over leg positions: for ordering o, input slot k
   * < n_legs is external leg orderings[o][k], and A_o is the template's
   * amplitude combination (every jamp row identical). */
  int32_t n_orderings;
  const int8_t* orderings;            /* [n_orderings][n_legs] permutations of 0..n_legs-1 */
  /* Flow map for an ordering template, or NULL: flow f's jamp is
   * J_f = sum_o flow_map[f][o] A_o (e.g. the Kleiss-Kuijf expansion of the
   * (n-1)! trace-basis partial amplitudes over the (n-2)! evaluated ones).
   * NULL means J_o = A_o and n_flows = n_orderings.  Every row needs at least
   * one non-zero entry.  Templates with n_flows >= 32 contract the colour
   * matrix on MFMA (Sec. 5.4's colour sum as a batched dense product). */
  const int8_t* flow_map;             /* [n_flows][n_orderings] */
  /* Phase space of generated events: n_ps_nodes = 0 for RAMBO (flat massless
   * n-body, constant weight; every final leg must then be massless), else the
   * resonance tree ps_nodes[0 .. n_ps_nodes-1]
   * (node 0 = the collision; every final leg and every other node the daughter
   * of exactly one node) with the window factor ps_window (> 0; the paper's
   * default is 20).  Part of the kernel's structure (compiled in). */
  int32_t n_ps_nodes;
  const heget_ps_node* ps_nodes;
  double ps_window;
  /* Hadronic collision (the paper's Appendix A, parton densities set to 1):
   * ps_hadron_ymax > 0 makes node 0 of the tree a parton collision at a hadron
   * collider whose energy is the sqrt_s of eval / integrate.  Node 0's two
   * daughters get rapidities flat in [-ymax, ymax], the first daughter
   * ln(m^2 + pT^2) flat from pT = ps_hadron_ptmin (> 0 for a massless daughter)
   * to the kinematic limit and a flat azimuth, the second the balancing pT;
   * x_a, x_b = sum (E +- p_z) / sqrt_s, the event's weight 0 unless both are
   * below 1.  dSigma_2 = (2 pi / S) dy_1 dy_0 dpT^2 / (4 pi)^2 dphi / (2 pi); the
   * partonic flux 1 / (2 s_hat) joins the per-event weight.  0: the tree's
   * collision at fixed sqrt_s (rest frame).  Part of the kernel's structure. */
  double ps_hadron_ymax;
  double ps_hadron_ptmin;
  /* Colour form of the compiled kernel: 0 dense (the colour matrix as given;
   * on MFMA for templates with n_flows >= 32), 1 compressed (Sec. 5.4: each
   * row's entries grouped by their distinct colour factors, one multiplication
   * per factor and row, on VALU; FP64 kernels of bases with n_flows >= 32 keep
   * the dense MFMA form).  Part of the kernel's structure. */
  int32_t colour_form;
  /* Division of the amplitude program (Sec. 5.3): 0 fused (one kernel), 1 split
   * (ordering templates only: the orderings' amplitudes in one kernel, written
   * to the handle's workspace, the colour form and the weights in a second one,
   * the two launched one after the other for each round of resident blocks).
   * Part of the kernel's structure. */
  int32_t division;
} heget_process_ir;

typedef struct heget_process* heget_process_t;

typedef struct {
  double sigma_gev2, err_gev2;   /* cross section and its Monte Carlo error, GeV^-2 */
  double sigma_pb, err_pb;       /* the same in pb ((hbar c)^2 = 0.3893793721e9 pb GeV^2) */
  double sum_w, sum_w2;          /* sum of weights and of squared weights */
  int64_t n_generated, n_accepted;
} heget_result;

/* The process as the paper's amplitude generator hands it over (Sec. 5.1-5.2:
 * the HEGET call sequence converted one to one from the HELAS calls, the
 * process's particles, graphs and colour bases; Sec. 4: the external-line and
 * vertex functions; Sec. 5.4: the colour matrix).
 * Validate the IR, derive the couplings and propagator table from ir->sm,
 * upload the helicity table and bind the compiled kernel whose structure
 * (legs, calls, jamps, colour matrix) matches the IR.  prec selects FP64 or the
 * mixed path (FP32 wavefunctions, vertex chain and colour sum; FP64 momenta,
 * propagator denominators and reductions).  *out receives the handle.
 * Errors: HEGET_E_INVALID (null pointers), HEGET_E_IR (malformed IR),
 * HEGET_E_UNSUPPORTED (no kernel compiled for this structure; or HEGET_MIXED for a
 * process whose colour form runs on MFMA, switched off after unexplained GPU
 * faults of those mixed kernels), HEGET_E_OOM, HEGET_E_HIP.  heget_eval never
 * allocates. */
heget_status heget_process_create(const heget_process_ir* ir, heget_precision prec, heget_process_t* out);

/* Release the handle and its device tables (synchronises the device first).
 * No passage of the paper: resource release only. */
heget_status heget_process_destroy(heget_process_t p);

/* The integrand of Sec. 2 at n phase-space points: for each point the squared
 * amplitude summed over the helicities and colour indices of every external
 * particle (Sec. 2, the LO partonic cross-section formula; the per-point
 * evaluation one thread each, Sec. 3), from the external wavefunctions and
 * vertex chain of Sec. 4 and the colour matrix of Sec. 5.4.
 * Evaluate n events on `stream` (asynchronous; hipStream_t passed as void*).
 * momenta_in: device FP64 SoA [n_legs][4][n] physical momenta (E, px, py, pz),
 *   or NULL to generate them: incoming partons along +z / -z with energy
 *   sqrt_s / 2 each, final state by RAMBO from Philox4x32-10 with key `seed`
 *   and event counters counter_offset .. counter_offset + n - 1.
 * me2_out: device FP64 [n]: helicity- and colour-summed |M|^2 (no averaging,
 *   no symmetry factor); events failing the IR's cut get 0.  May be NULL.
 * momenta_out: device FP64 SoA [n_legs][4][n] of the momenta used, or NULL.
 * n = 0 is a no-op.  Errors: HEGET_E_INVALID, HEGET_E_HIP. */
heget_status heget_eval(heget_process_t p, int64_t n, const double* momenta_in, uint64_t seed,
                        uint64_t counter_offset, double sqrt_s, double* me2_out, double* momenta_out,
                        void* stream);

/* Phase-space generation alone: the momenta heget_eval would generate for
 * (seed, counter_offset .. counter_offset + n - 1, sqrt_s), written to the
 * device FP64 SoA momenta_out [n_legs][4][n] (the Philox -> phase-space step of
 * the integrand, Sec. 3; 32 bytes per leg per event, an HBM-bound kernel), and,
 * if weights_out (device FP64 [n]) is not NULL, each event's phase-space weight
 * dPhi_n (GeV^(2n-4); RAMBO: the constant n-body volume; resonance tree: the
 * product of the tree's two-body volumes and mapping Jacobians, 0 where a
 * window is empty).  Asynchronous on `stream`.  n = 0 is a no-op (the outputs
 * may then be NULL).  Errors: HEGET_E_INVALID (null handle, null momenta_out
 * with n > 0, n < 0, sqrt_s <= 0), HEGET_E_UNSUPPORTED (RAMBO with more than 10
 * final-state legs), HEGET_E_HIP. */
heget_status heget_generate(heget_process_t p, int64_t n, uint64_t seed, uint64_t counter_offset, double sqrt_s,
                            double* momenta_out, double* weights_out, void* stream);

/* The counter-based random numbers alone (the first step of every generated
 * event; not in the paper, which seeds a per-thread xorshift generator: the
 * counter-based Philox4x32-10 of Salmon et al., SC'11, makes any event
 * reproducible from (seed, event index)).  Event i (counter counter_offset + i)
 * uses counter (i_lo, i_hi, j, 0) and key (seed_lo, seed_hi) for its block j,
 * and block j gives the uniforms 2 j and 2 j + 1: u = (floor(x / 2^12) + 1/2)
 * 2^-52 for the 64-bit words x = w0 2^32 + w1 and x = w2 2^32 + w3, exact in
 * FP64 and strictly inside (0, 1).  These are the uniforms heget_eval's RAMBO
 * and resonance-tree generators draw (RAMBO: 4 per final particle, in the
 * order cos theta, phi, and the two factors of the energy).  u_out: device
 * FP64 SoA [n_u][n], u_out[k * n + i] = uniform k of event i; written
 * asynchronously on `stream`.  n = 0 is a no-op.  Errors: HEGET_E_INVALID
 * (n < 0, n_u outside 1 .. 64, null u_out with n > 0), HEGET_E_HIP. */
heget_status heget_uniforms(uint64_t seed, uint64_t counter_offset, int64_t n, int32_t n_u, double* u_out,
                            void* stream);

/* The LO partonic cross section of Sec. 2 (the flux, spin and colour averages
 * and the integral of the summed squared amplitude over the n-body phase
 * space) as a plain Monte Carlo estimate over points generated one per thread
 * with no retry (Sec. 3); the paper integrates with BASES on the GPU (Sec. 6),
 * whose adaptive grid heget_integrate_adaptive provides.
 * Monte Carlo cross section from n events generated from `seed` (counters
 * 0 .. n-1) by the process's phase space (RAMBO or its resonance tree):
 * sigma = (1/N) sum_i w_i with w_i = dPhi_n,i * pass_i * F_i / (2 lambda^(1/2) N_pol n_a n_b S),
 * lambda^(1/2) = lambda^(1/2)(s, m_a^2, m_b^2) the flux of the incoming legs (s when
 * both are massless) and N_pol their polarisation states (2 per fermion or
 * massless vector, 3 per massive vector, 1 per scalar), reduced on the device
 * in a fixed order.  Synchronises
 * `stream`; fills *out.  The handle keeps a small buffer of per-block partial
 * sums (24 bytes per 256 events), allocated on the first call and grown when a
 * larger n arrives, and 24 bytes of pinned host memory for the reduced sums;
 * calls on one handle must not overlap.
 * Errors: HEGET_E_INVALID, HEGET_E_OOM, HEGET_E_HIP. */
heget_status heget_integrate(heget_process_t p, int64_t n, double sqrt_s, uint64_t seed, heget_result* out,
                             void* stream);

/* heget_integrate as one stage of a pipeline: the Monte Carlo event loop of
 * Sec. 6 with the host queueing batch after batch while the device works.
 * Enqueues on `stream` the same kernels, counters and fixed-order reduction as
 * heget_integrate and returns without waiting.  Once the stream has passed the
 * call, sums_out[0..2] hold sum w, sum w^2 and the accepted count (as a
 * double), bit for bit the sums heget_integrate reduces;
 * heget_result_from_sums turns them into the heget_result heget_integrate
 * fills.  sums_out: 3 doubles of device memory, or of pinned host memory,
 * owned by the caller and kept until the stream has passed the call.  Calls on
 * one handle share its per-block partial sums: make them on one stream, which
 * orders them (calls on two streams at once race).  A call with n above every
 * earlier call's grows that buffer, after waiting for `stream`.
 * Errors: HEGET_E_INVALID (null handle or sums_out, n < 2, sqrt_s <= 0,
 * sums_out in pageable host memory, i.e. not known to HIP), HEGET_E_OOM,
 * HEGET_E_HIP (a launch failed; the call enqueues nothing more). */
heget_status heget_integrate_async(heget_process_t p, int64_t n, double sqrt_s, uint64_t seed, double* sums_out,
                                   void* stream);

/* The cross section of n events from the three sums of heget_integrate_async
 * (host memory): sigma = sum w / n, its Monte Carlo error
 * sqrt((sum w^2 / n - sigma^2) / (n - 1)), in GeV^-2 and in pb
 * (hbar c)^2 = 0.3893793721e9 pb GeV^2).  Errors: HEGET_E_INVALID (null
 * pointer, n < 2). */
heget_status heget_result_from_sums(const double* sums, int64_t n, heget_result* out);

/* heget_integrate for callers that cannot allocate (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * kernels, counters, reduction order and result as heget_integrate (bit for
 * bit), with the per-block partial sums and the reduced sums in a fixed scratch
 * array of the library instead of buffers of the handle; the result is read
 * back into host memory of the call itself.  The call allocates nothing and
 * calls no allocating routine.  n is at most HEGET_NOALLOC_MAX_EVENTS (the
 * scratch holds 24 bytes per 256 events: 6 MiB per GPU, held until the process
 * ends).  Every call on one GPU shares that GPU's scratch: calls that overlap
 * on one GPU (from several threads or streams) race and must not be made.
 * The scratch's address is looked up once per device, by heget_process_create
 * or by this call's first use on a device.  Synchronises `stream`; fills *out.
 * Errors: HEGET_E_INVALID (null handle or out, n < 2, n above the limit,
 * sqrt_s <= 0), HEGET_E_HIP. */
#define HEGET_NOALLOC_MAX_EVENTS (INT64_C(1) << 26)
heget_status heget_integrate_noalloc(heget_process_t p, int64_t n, double sqrt_s, uint64_t seed,
                                     heget_result* out, void* stream);

/* Adaptive Monte Carlo integration (the role of the BASES integrator in the
 * paper's runs, Sec. 1 and 6): `iterations` passes of n events each, iteration
 * k drawing counters k n .. (k + 1) n - 1 from `seed`; the uniforms of the
 * process's resonance-tree phase space go through a VEGAS grid (G. P. Lepage,
 * J. Comput. Phys. 27 (1978) 192) of `bins` bins per dimension, uniform at the
 * start and refined after every pass from the sums of w^2 per bin (smoothing
 * over neighbouring bins, compression ((x - 1) / ln x)^1.5, equal shares per new
 * bin).  per_iteration (host, [iterations], may be NULL) gets each pass's
 * result; *combined the inverse-variance average (a pass with zero error takes
 * no weight; if every pass has zero error, the plain mean with error 0;
 * n_generated, n_accepted, sum_w, sum_w2 summed over the passes); *chi2_per_dof (may be NULL) the
 * passes' consistency; grid_out (host, [dims][bins + 1], may be NULL) the
 * final grid.  The passes run back to back on `stream` (the grid refined on
 * the device between them); the call synchronises `stream` once, at the end.
 * The handle keeps the device buffers (about 9 + dims bytes per event),
 * allocated on the first call and grown when a larger n arrives; calls on one
 * handle must not overlap.  Errors: HEGET_E_INVALID (null
 * handle or combined, n < 2, iterations < 1, bins outside 2 .. 32, sqrt_s <= 0),
 * HEGET_E_UNSUPPORTED (a process without a resonance tree), HEGET_E_OOM,
 * HEGET_E_HIP. */
heget_status heget_integrate_adaptive(heget_process_t p, int64_t n, int32_t iterations, int32_t bins,
                                      double sqrt_s, uint64_t seed, heget_result* per_iteration,
                                      heget_result* combined, double* chi2_per_dof, double* grid_out,
                                      void* stream);

/* Uniforms per event of the process's phase space that an adaptive grid maps
 * (the grid's dimensions; 0 for RAMBO processes), or -1 for a null handle. */
int32_t heget_process_grid_dims(heget_process_t p);

/* Number of helicity combinations the handle sums (after heget_filter_helicities). */
int32_t heget_process_n_helicities(heget_process_t p);

/* Drop helicity combinations whose colour-summed |M|^2 is below rel_threshold
 * times the largest one on every one of n_probe generated events (an exact
 * zero gives 0 on every event).  Synchronous; uses the handle's own kernel.
 * Returns the number kept in *n_kept.  Errors: HEGET_E_INVALID, HEGET_E_HIP. */
heget_status heget_filter_helicities(heget_process_t p, int64_t n_probe, uint64_t seed, double sqrt_s,
                                     double rel_threshold, int32_t* n_kept);

/* Thread-local message describing the last non-OK status ("" if none). */
const char* heget_last_error(void);

/* ------------------------------------------------------------------ serving
 * A request loop over resident processes: requests heget_integrate(process,
 * n, sqrt_s, seed) arrive at any time from any thread, are admitted in arrival
 * order while their device footprint fits a fixed arena, and run as fused
 * launches (several requests of one process in one persistent kernel, replayed
 * from a HIP graph captured at creation), several launches at once on their
 * own streams.  A request split over several launches keeps the Philox
 * counters, partial-sum slots and reduction order of heget_integrate of that
 * request alone: its result is bit-identical to that call on the same handle,
 * whatever else is in flight.  The process handles stay owned by the caller,
 * must outlive the server, and must not be used for heget_filter_helicities
 * while the server exists (the server captures their tables at creation). */
typedef struct heget_server* heget_server_t;

typedef struct {
  int32_t n_processes;
  const heget_process_t* processes;  /* [n_processes], each with its own precision */
  int64_t arena_bytes;               /* device memory for requests in flight (>= 1 MiB) */
  int32_t slots_per_process;         /* concurrent fused launches per process, 1..8 */
  int32_t max_batch_blocks;          /* 256-event blocks per fused launch */
  int32_t max_chunk_blocks;          /* blocks of one request per fused launch */
} heget_server_config;

typedef struct {
  int64_t requests_submitted, requests_done;
  int64_t launches, segments, events;  /* fused launches, request segments in them, events run */
  int64_t arena_high_water;            /* bytes */
  int32_t max_busy_slots;              /* most fused launches in flight at once */
} heget_server_stats;

/* Allocates the arena, captures one graph per (process, slot) and starts the
 * scheduler thread on the current device.
 * Errors: HEGET_E_INVALID (bad configuration), HEGET_E_OOM, HEGET_E_HIP. */
heget_status heget_server_create(const heget_server_config* cfg, heget_server_t* out);

/* Queue a request; returns at once with its ticket.  Footprint: 24 bytes per
 * 256 events, plus 8 bytes per event if me2_host is given (then the request's
 * |M|^2 per event, as heget_eval would give it, is copied into me2_host[n]
 * before the request completes; the buffer must stay valid until then).
 * Errors: HEGET_E_INVALID (bad index, n < 2, sqrt_s <= 0, footprint larger
 * than the arena, server shutting down). */
heget_status heget_server_submit(heget_server_t s, int32_t process, int64_t n, uint64_t seed, double sqrt_s,
                                 double* me2_host, uint64_t* ticket);

/* Result of a request: with wait != 0 blocks until it is done.  Sets *done;
 * when done, fills *out and the submit-to-completion time *latency_s (may be
 * NULL) and forgets the ticket.  Errors: HEGET_E_INVALID (unknown ticket), or
 * the request's own failure (HEGET_E_HIP). */
heget_status heget_server_poll(heget_server_t s, uint64_t ticket, int32_t wait, heget_result* out,
                               double* latency_s, int32_t* done);

/* Counters since creation. */
heget_status heget_server_stats_get(heget_server_t s, heget_server_stats* out);

/* Runs every queued request to completion, stops the scheduler and frees the
 * server (not the process handles).  Tickets not yet polled are dropped. */
heget_status heget_server_destroy(heget_server_t s);

#ifdef __cplusplus
}
#endif
#endif
