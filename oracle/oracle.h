/* Oracle C interface (test infrastructure only).
 *
 * A plain, slow FP64 CPU implementation of what the per-event amplitude path
 * computes: counter-based uniforms, RAMBO momenta, the generation cut, and the
 * helicity- and colour-summed squared matrix element F = sum_hel sum_col |M|^2
 * for each process, written from textbook Feynman rules derived from the
 * paper's Lagrangians (Sec. 4.2) with explicit Dirac matrices.  Gluon processes
 * use an independent colour-ordered Berends-Giele recursion.
 *
 * Only tests, the smoke check and the benchmark's CPU-baseline leg may load
 * this library.  It shares no code with the product path.
 *
 * Momenta layout for every call: array-of-structures [n_events][n_legs][4],
 * physical momenta (E, px, py, pz); legs ordered as documented per process.
 */
#ifndef HEGET_ORACLE_H
#define HEGET_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
  double alpha;    /* QED coupling (1/128) */
  double sw2;      /* sin^2 theta_W */
  double mz, wz;   /* Z mass and width */
  double mw, ww;   /* W mass and width (ignored when cms != 0) */
  double mt, wt;   /* top mass and width */
  double mh, wh;   /* Higgs mass and width */
  double alpha_s;  /* strong coupling */
  double mb_yuk;   /* b mass used in the Yukawa coupling only (b is massless kinematically) */
  int cms;         /* 1: complex-mass scheme for W/Z, mu_W^2 = c_W^2 mu_Z^2 */
  int gauge_leg;   /* -1, or the index of a vector leg whose polarisation is replaced by k/k^0 */
} or_params;

/* process identifiers */
enum {
  OR_EE_MUMU = 0,       /* e-(in,+z) e+(in,-z) -> mu- mu+  via gamma + Z */
  OR_GG_TT_6F = 1,      /* g g -> t tbar -> (b e+ nu_e)(bbar mu- nu_mu~) legs g g b e+ ve bbar mu- vm~ */
  OR_GG_4G = 2,         /* g g -> g g g g (Berends-Giele) */
  OR_UD_UDHH_4B = 3,    /* u d -> u d H H, H -> b bbar; legs u d u d b bbar b bbar */
  OR_GG_GG = 10,        /* g g -> g g (Berends-Giele) */
  OR_GG_GGG = 11,       /* g g -> g g g (Berends-Giele) */
  OR_UU_TT = 12,        /* u ubar -> t tbar, stable tops: legs u ubar t tbar */
  OR_GG_TT = 13,        /* g g -> t tbar, stable tops: legs g g t tbar */
  OR_UU_UUHH_4B = 14,   /* u u -> u u H H, H -> b bbar (Fermi-sign check) */
  OR_WW_HH = 16,        /* W- W+ -> H H with on-shell external W (unitarity check) */
  OR_ZZ_HH = 17,        /* Z Z -> H H with on-shell external Z */
  OR_UD_UDHHH = 4,      /* u d -> u d H H H by W W and Z Z fusion; legs u d u d H H H */
  OR_WW_HHH = 18,       /* W- W+ -> H H H with on-shell external W (unitarity check) */
  OR_ZZ_HHH = 19,       /* Z Z -> H H H with on-shell external Z */
  OR_WW_WW = 20,        /* W- W+ -> W- W+ with on-shell external W; legs W- W+ W- W+ */
  OR_GG_5G = 21,        /* g g -> g g g g g (Berends-Giele; colour matrix by Fierz expansion) */
  /* u ubar -> t tbar + n gluons by Feynman diagrams; legs u ubar t tbar g ... */
  OR_UU_TTG = 22, OR_UU_TTGG = 23, OR_UU_TTGGG = 24,
  OR_UU_TT_DIAG = 25    /* n = 0 through the same diagram code (compare OR_UU_TT) */
};

int or_nlegs(int proc);

/* Philox4x32 with 10 rounds (Salmon et al., SC'11). */
void or_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);

/* n_u uniforms in (0,1) for event index `event`: block j uses counter
 * (event_lo, event_hi, j, 0) and key (seed_lo, seed_hi); each block yields two
 * uniforms u = (floor(x / 2^12) + 1/2) 2^-52 from x = w0 2^32 + w1 and
 * x = w2 2^32 + w3 (exact in FP64, strictly inside (0,1)). */
void or_uniforms(uint64_t seed, uint64_t event, int n_u, double* u);
/* the same for events counter_offset .. counter_offset + n_events - 1: u[i][n_u] */
void or_uniforms_bulk(uint64_t seed, uint64_t counter_offset, int64_t n_events, int n_u, double* u);

/* RAMBO (Kleiss, Stirling, Ellis 1986): n massless momenta in the centre-of-mass
 * frame at energy sqrt_s from 4n uniforms (per particle: cos theta, phi, two
 * energies).  Writes p[n][4]; returns the constant phase-space weight. */
double or_rambo(double sqrt_s, int n, const double* u, double* p);

/* Closed-form massless n-body phase-space volume. */
double or_phase_space_volume(double sqrt_s, int n);

/* Full event generation for a 2 -> n_out process: incoming momenta along +-z,
 * then RAMBO outgoing momenta.  mom[n_events][2 + n_out][4]. */
void or_generate(uint64_t seed, uint64_t counter_offset, int64_t n_events, int n_out, double sqrt_s,
                 double* mom);

/* Generation cut for g g -> 4g: every final gluon pT > pt_min and every final
 * pair Delta R > dr_min.  mom as above (6 legs).  Writes 1 / 0 per event. */
void or_cut_gluons(int64_t n_events, int n_legs, const double* mom, double pt_min, double dr_min,
                   int32_t* pass);

/* Helicity- and colour-summed |M|^2 (no averaging, no symmetry factor) per event. */
int or_eval(int proc, const or_params* prm, int64_t n_events, const double* mom, double* me2,
            int n_threads);

/* Conditioning of the diagram sum per event (processes with a diagram list):
 * kappa = sqrt( sum_{hel,col} (sum_d |c_d M_d|)^2 / sum_{hel,col} |sum_d c_d M_d|^2 ),
 * the factor by which rounding errors of the individual diagrams are amplified
 * in the relative error of F.  kappa >= 1; 1 means no cancellation. */
int or_condition(int proc, const or_params* prm, int64_t n_events, const double* mom, double* kappa,
                 int n_threads);

/* Amplitude for one helicity combination and one explicit colour assignment
 * (processes with quarks: 1, 3, 14).  Colour indices: gluons 0..7, quarks 0..2,
 * one per leg (ignored for colourless legs).  out = {re, im}. */
int or_amp_colour(int proc, const or_params* prm, const double* mom, const int* hel, const int* col,
                  double* out);

/* Per-helicity colour-summed |M|^2 for one event: out[n_hel] in the order of
 * the helicity table returned by or_helicities. */
int or_me2_per_helicity(int proc, const or_params* prm, const double* mom, double* out);
int or_helicities(int proc, int* table /* [n_hel][n_legs] or NULL */);

/* Colour-summed |M|^2 for one explicit helicity vector (vector legs also accept
 * 4 = gauge vector k/k^0 and 10+alpha = unit vector along axis alpha). */
int or_me2_hel(int proc, const or_params* prm, const double* mom, const int* hel, double* out);

/* Colour-ordered partial amplitude A(1, sigma) of the n-gluon process (n = 4..6)
 * for one helicity combination; order[] lists all n legs starting with 0.
 * Legs 0, 1 are incoming.  out = {re, im}. */
int or_gluon_partial(int n, const or_params* prm, const double* mom, const int* hel, const int* order,
                     double* out);

/* Colour matrix C[sigma][tau] = sum over all gluon colours of
 * Tr(T^a1 T^a_sigma2 ...) conj(Tr(T^a1 T^a_tau2 ...)), brute force over SU(3);
 * orderings enumerated as the lexicographic permutations of legs 1..n-1. */
int or_gluon_colour_matrix(int n, double* C);

/* The same matrix by Fierz expansion and closed-loop counting (n = 3 .. 8);
 * the matrix the oracle uses from 7 gluons on. */
int or_gluon_colour_matrix_fierz(int n, double* C);

/* Spin-summed |M|^2 from Dirac traces with completeness relations (no spinors):
 * proc OR_UU_TT or OR_GG_TT, colour summed. */
int or_trace_me2(int proc, const or_params* prm, const double* mom, double* out);

/* Weighted cross-section pieces: w_i = phase-space weight * pass_i *
 * factor * F_i, where factor = 1/(2 s) * 1/4 * 1/(n_a n_b) * 1/S.  Weights are
 * returned per event so the caller can sum them exactly. */
int or_weights(double phase_space_weight, double factor, int64_t n_events, const double* me2,
               const int32_t* pass, double* w);

/* Tree-level two-body decay width (GeV) from the oracle's W-fermion vertex,
 * spinors and massive polarisation vectors, spin-summed and averaged:
 * which 0 = W+ -> e+ nu_e (massless leptons), 1 = t -> b W+ (massless b).
 * Returns -1 for an unknown `which`. */
int or_decay_width(int which, const or_params* prm, double* out);

/* Self-checks of the building blocks (Dirac equation, completeness, helicity,
 * polarisation orthogonality); returns the largest violation found. */
double or_selfcheck_spinors(const double* p, double m);

#ifdef __cplusplus
}
#endif
#endif
