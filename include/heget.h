/*
 * heget.h - C ABI of the MI355X (gfx950) tree-level QCD matrix-element library.
 *
 * The library evaluates, for many phase-space points at once, the squared
 * tree-level matrix element of a massless QCD process
 *
 *     |M|^2 = 1/4 sum_lambda  sum_{alpha,beta} J_alpha N_alpha,beta J_beta^*
 *
 * averaged over the spins and colours of the two initial partons and summed
 * over those of the final ones, as defined in section 2.1 of Hagiwara et al.,
 * "Calculation of HELAS amplitudes for QCD processes using graphics processing
 * unit (GPU)" (arXiv:0909.5257): eq. (matrix-element) for the diagram sum,
 * eq. (color-amplitude) for the colour-basis amplitudes J, eq. (color-matrix)
 * for N, eq. (color-averaged-amplitude) for the colour sum and the helicity
 * sum-average defined right after it.  The identical-particle factor that the
 * paper puts on the phase space (remark after eq. phase-space) is NOT applied.
 *
 * Supported processes are those of the paper's eq. (processes) / Table 1 for
 * which kernels were generated at build time; heget_num_processes and
 * heget_process_spec list them.
 *
 * Status codes: every entry point returns HEGET_OK or an error code and never
 * throws.  Argument errors are detected before any device work is queued.
 * Device errors of asynchronous work surface as HEGET_E_DEVICE from a later
 * call or from the caller's stream synchronisation.
 */
#ifndef HEGET_H
#define HEGET_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct heget_process* heget_process_t;

typedef enum {
  HEGET_OK = 0,
  HEGET_E_INVALID_ARG = 1,          /* null / misaligned pointer, bad size, bad alpha_s */
  HEGET_E_UNSUPPORTED_PROCESS = 2,  /* spec not parsable or no kernel generated for it */
  HEGET_E_OUT_OF_MEMORY = 3,        /* device allocation of process state failed */
  HEGET_E_DEVICE = 4                /* HIP runtime error (launch or copy) */
} heget_status;

typedef enum {
  HEGET_FP64 = 0,   /* every step in float64 */
  HEGET_MIXED = 1   /* wavefunctions, currents and amplitudes in float32; momenta,
                       invariants, JAMP accumulation and colour sum in float64 */
} heget_precision;

/* Create a process handle.
 *   spec      process string "a b > f1 f2 ...", partons g, u, u~ separated by
 *             blanks, e.g. "g g > g g g g", "u u~ > g g g g g", "u u > u u g g g".
 *             Leg order of the momenta is the order written here.
 *   precision HEGET_FP64 or HEGET_MIXED.
 *   out       receives the handle; the library owns the process state (the
 *             colour matrix uploaded to the current HIP device) until
 *             heget_destroy_process.
 * The handle is bound to the HIP device current at creation and is immutable,
 * so concurrent heget_matrix_elements calls on different streams are safe.
 * Errors: HEGET_E_INVALID_ARG (null spec/out or bad precision),
 * HEGET_E_UNSUPPORTED_PROCESS, HEGET_E_OUT_OF_MEMORY, HEGET_E_DEVICE. */
heget_status heget_create_process(const char* spec, heget_precision precision, heget_process_t* out);

/* Static properties of a process (Table 1 counts of the paper for the
 * supported processes).  n_helicities counts the helicity configurations that
 * are not structural zeros of massless-quark chirality.  Any pointer may be
 * NULL.  Errors: HEGET_E_INVALID_ARG for a NULL handle. */
heget_status heget_process_info(heget_process_t p, int* n_ext, int* n_diagrams, int* n_colours,
                                int* n_helicities);

/* Spin/colour averaged |M|^2 for n_events phase-space points.
 *   momenta  DEVICE pointer, float64, layout [n_events][n_ext][4] with
 *            components (E, px, py, pz) in GeV; initial partons carry their
 *            physical incoming momenta and final ones their outgoing momenta;
 *            all partons massless.  16-byte aligned.  Read only.
 *   n_events number of points, 0 <= n_events <= 2^36; 0 queues nothing.
 *   alpha_s  strong coupling (g_s^2 = 4 pi alpha_s), finite and > 0.
 *   me2      DEVICE pointer, float64 [n_events], written.
 *   stream   hipStream_t to queue the work on (NULL: the default stream).
 * Buffers are owned by the caller and must stay valid until the queued work
 * completes.  The call is asynchronous.
 * Errors: HEGET_E_INVALID_ARG (detected synchronously, nothing queued),
 * HEGET_E_DEVICE (launch failure). */
heget_status heget_matrix_elements(heget_process_t p, const double* momenta, int64_t n_events, double alpha_s,
                                   double* me2, void* stream);

/* One term of the helicity sum per event: the Monte Carlo helicity mode of the
 * paper's program structure (section 3.2, steps 2 and 4), where each phase-space
 * point carries one helicity configuration drawn on the host and only that
 * configuration's colour-summed |J|^2 (eq. color-averaged-amplitude) is
 * evaluated.
 *   momenta, n_events, alpha_s, me2, stream  as for heget_matrix_elements.
 *   helicity DEVICE pointer, int32 [n_events], read only: a bit pattern h in
 *            [0, 2^n_ext) with bit i set when leg i has helicity +1 and clear
 *            when it has -1 (the helicity of an incoming parton as it enters).
 * me2[e] = 1/4 * sum_{alpha,beta} J_alpha(h_e) N_alpha,beta J_beta(h_e)^*, so that the
 * sum over all 2^n_ext patterns equals heget_matrix_elements and 2^n_ext * me2
 * is an unbiased estimate of it for uniformly drawn h.  Structural zeros give
 * exactly 0; an h outside [0, 2^n_ext) gives NaN for that event.
 * For processes with several quark-chirality patterns (two quark lines) and
 * n_events < 2^31 the events are first sorted by pattern on the device, with
 * work space of 16 bytes per event plus the sort's own taken from and returned
 * to the device's stream-ordered pool; results are written in event order.
 * Errors: as heget_matrix_elements, plus HEGET_E_INVALID_ARG for a NULL
 * helicity pointer and HEGET_E_OUT_OF_MEMORY if the sort's work space fails. */
heget_status heget_matrix_elements_helicity(heget_process_t p, const double* momenta, const int32_t* helicity,
                                            int64_t n_events, double alpha_s, double* me2, void* stream);

/* Exact colour matrix N_alpha,beta of eq. (color-matrix), including the
 * 1/(n_a n_b) colour average: N = num / den element-wise, row-major K x K, in
 * the colour basis of eq. (color-amplitude) (single traces with leg 0 first for
 * gluons, chains for one quark line, chain pairs sharing one summed adjoint
 * index for two quark lines; orderings in lexicographic permutation order).
 *   n_colours receives K (required).
 *   num, den, values  HOST arrays of K*K entries, each may be NULL.
 * Errors: HEGET_E_INVALID_ARG for a NULL handle or n_colours. */
heget_status heget_color_matrix(heget_process_t p, int* n_colours, int64_t* num, int64_t* den, double* values);

/* Algorithmic floating-point operations per event: every evaluated helicity
 * configuration's external wavefunctions, each shared current once, every
 * diagram amplitude, the JAMP accumulation and the colour quadratic form,
 * counted by the generator from the routines it emits (roofline numerator).
 * Errors: HEGET_E_INVALID_ARG for a NULL argument. */
heget_status heget_process_flops(heget_process_t p, int64_t* flops_per_event);

/* One item of a fused batch: a process handle and its own device buffers,
 * with the layouts of heget_matrix_elements. */
typedef struct {
  heget_process_t process;
  const double* momenta;   /* DEVICE [n_events][n_ext][4], 16-byte aligned */
  int64_t n_events;
  double* me2;             /* DEVICE [n_events] */
} heget_batch_item;

/* Evaluate several processes of uneven sizes as one unit of work (the per-item
 * quantity is that of heget_matrix_elements).  The call forks from `stream`
 * onto a pool of library-owned HIP streams (default priority), places the
 * items on them longest-first by their flop count (heget_process_flops x
 * n_events) and joins back into `stream`, so small and large processes run
 * concurrently.  With use_graph != 0 the whole fork/launch/join sequence is
 * captured once into a hipGraph, cached by the exact item list (handles,
 * pointers, sizes, alpha_s) and replayed on later identical calls.
 *   items    HOST array of n_items entries; all handles on the current device.
 *   stream   hipStream_t the batch is ordered after and before (NULL: default).
 * Every item's buffers must stay valid until the batch completes; items must
 * not alias each other's me2.  Asynchronous like heget_matrix_elements.
 * Errors: HEGET_E_INVALID_ARG (any item invalid: nothing is queued),
 * HEGET_E_DEVICE (stream/graph/launch failure). */
heget_status heget_matrix_elements_batch(const heget_batch_item* items, int n_items, double alpha_s,
                                         int use_graph, void* stream);

/* Precision of the colour contraction in heget_colour_quadratic_form. */
typedef enum {
  HEGET_COLOUR_FP64 = 0,       /* float64 on the matrix cores */
  HEGET_COLOUR_FP32 = 1,       /* float32 operands on the matrix cores, float32 accumulate */
  HEGET_COLOUR_BF16X3 = 2,     /* bf16 hi/lo split, three matrix-core products, float32 accumulate */
  HEGET_COLOUR_FP64_VALU = 3   /* float64 on the vector ALUs (n_colours <= 128) */
} heget_colour_mode;

/* Colour quadratic form of eq. (color-averaged-amplitude) for many amplitude
 * vectors at once, written as a GEMM: with the real and imaginary parts of J
 * as separate rows X (2R x K), Y = X N and q_r = X_2r.Y_2r + X_2r+1.Y_2r+1.
 * This is the colour step of the paper in its own basis (section 3.3: eq.
 * color-matrix, Table 3), offered for precision and speed studies of the
 * contraction (the process kernels do the same sum in an exactly reduced
 * colour space).
 *   n_colours     K > 0 (K > 128 only for the three matrix-core modes).
 *   colour_matrix DEVICE float64 K x K, symmetric (e.g. heget_color_matrix values).
 *   jamp          DEVICE float64 [rows][2][K]: Re J then Im J of each row.
 *   rows          number of amplitude vectors R, 0 <= R < 2^30.
 *   mode          HEGET_COLOUR_FP64 / _FP32 / _BF16X3 / _FP64_VALU.
 *   q             DEVICE float64 [rows], written.
 *   stream        hipStream_t (NULL: default stream).
 * For K <= 128 hand-written kernels read J once and need no work space.  For
 * K > 128 the product is a library GEMM whose work space (at most 1.25 times
 * the bytes of jamp) is taken from and returned to the device's default
 * stream-ordered memory pool (the first such call on a device sets that pool
 * to keep up to 16 GiB of freed memory cached).  The row-wise dot is always
 * accumulated in float64 against the float64 J.
 * Errors: HEGET_E_INVALID_ARG, HEGET_E_OUT_OF_MEMORY, HEGET_E_DEVICE. */
heget_status heget_colour_quadratic_form(int n_colours, const double* colour_matrix, const double* jamp,
                                         int64_t rows, heget_colour_mode mode, double* q, void* stream);

/* ---------------------------------------------------------------------------
 * Phase space and integration on the device: steps 4 to 7 of the paper's
 * program structure (section 3.2) for a partonic collision at given sqrt(s)
 * (no parton densities).
 * ------------------------------------------------------------------------- */

/* Jet cuts of section 2.2 (eqs. cuts): every final parton must have
 * pT > pt_min (GeV) and |eta| < eta_max; if delta_r_min > 0 every pair must
 * also have Delta R = sqrt(d_eta^2 + d_phi^2) > delta_r_min (this replaces the
 * paper's relative-pT cut).  All comparisons are strict. */
typedef struct {
  double pt_min;
  double eta_max;
  double delta_r_min;
} heget_cuts;

/* Massless RAMBO (Kleiss, Stirling, Ellis, Comput. Phys. Commun. 40 (1986) 359):
 * turns 4 uniform numbers per final parton into n_final massless momenta in
 * the partonic centre-of-mass frame summing to (sqrt_s, 0, 0, 0).
 *   n_final   2..8.
 *   sqrt_s    DEVICE float64 [n_events], partonic energy per event (GeV).
 *   uniforms  DEVICE float64 [n_events][n_final][4] in (0, 1): per parton
 *             (cos theta = 2u0 - 1, phi = 2 pi u1, q0 = -log(u2 u3)).
 *   momenta   DEVICE float64 [n_events][n_final + 2][4], written: the two
 *             beams (sqrt_s/2)(1, 0, 0, +-1), then the finals; (E, px, py, pz).
 *   ps_weight DEVICE float64 [n_events] or NULL: the constant massless phase-
 *             space volume (2 pi)^(4-3n) (pi/2)^(n-1) s^(n-2) / ((n-1)! (n-2)!).
 * Asynchronous on stream.  Errors: HEGET_E_INVALID_ARG, HEGET_E_DEVICE. */
heget_status heget_rambo(int n_final, int64_t n_events, const double* sqrt_s, const double* uniforms,
                         double* momenta, double* ps_weight, void* stream);

/* Cut flags: pass[e] = 1 if event e's final partons (legs 2..n_ext-1 of
 * momenta [n_events][n_ext][4], DEVICE) pass *cuts (HOST struct), else 0.
 * pass is DEVICE uint8 [n_events].  Errors: HEGET_E_INVALID_ARG (n_ext outside
 * 4..10, non-finite cuts, eta_max <= 0), HEGET_E_DEVICE. */
heget_status heget_apply_cuts(int n_ext, int64_t n_events, const double* momenta, const heget_cuts* cuts,
                              uint8_t* pass, void* stream);

/* One integration step: RAMBO momenta from the uniforms, |M|^2 (summed over
 * helicities, or for one helicity pattern per event when helicity != NULL,
 * then scaled by 2^n_ext), the cuts, and the event weights of the partonic
 * cross section
 *     f_e = (hbar c)^2 * Phi_n(s_e) * |M|^2_e * pass_e / (2 s_e * S)   [pb]
 * with S the product of factorials of identical final partons (the factor
 * the paper puts on the phase space, remark after eq. phase-space), and their
 * sums.  The mean of f over the events estimates sigma-hat at sqrt_s.
 *   p, alpha_s   as for heget_matrix_elements; n_events >= 1.
 *   sqrt_s, uniforms, helicity  DEVICE inputs as for heget_rambo and
 *                heget_matrix_elements_helicity (helicity may be NULL).
 *   cuts         HOST struct.
 *   momenta      DEVICE float64 [n_events][n_ext][4], written (16-byte aligned).
 *   me2          DEVICE float64 [n_events], written: |M|^2 (helicity term x 2^n_ext
 *                is NOT applied here; it is the entry point's output).
 *   weight       DEVICE float64 [n_events], written: f_e.
 *   sums         DEVICE float64 [2], written: sum f_e and sum f_e^2, added in a
 *                fixed order, so they are identical on every run whenever me2 is.
 *                me2 is bit-reproducible for kernels that give each group of 64
 *                events one wave; kernels that share a group between several waves
 *                (large colour spaces, e.g. u u~ > g g g g g) add the waves'
 *                float64 colour-vector contributions in whatever order they
 *                arrive, so me2 and the sums can differ between runs by float64
 *                rounding (about 1e-16 relative).
 * Work space for block partials is taken and returned in stream order.
 * Errors: HEGET_E_INVALID_ARG, HEGET_E_OUT_OF_MEMORY, HEGET_E_DEVICE. */
heget_status heget_integrate_step(heget_process_t p, int64_t n_events, const double* sqrt_s, const double* uniforms,
                                  const int32_t* helicity, double alpha_s, const heget_cuts* cuts, double* momenta,
                                  double* me2, double* weight, double* sums, void* stream);

/* heget_integrate_step for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same kernels and results, but the block partial sums go to a fixed 2 MiB device
 * array that the library holds on every GPU it runs on until the process ends,
 * and nothing is allocated or freed.  With helicity != NULL the events are not
 * sorted by chirality pattern first (same results; two-quark-line processes run
 * slower).  Arguments and results as heget_integrate_step.
 *   n_events  1 .. 2^25 (33,554,432); larger batches return HEGET_E_INVALID_ARG.
 * All calls on one GPU share the array: calls that overlap in time on one GPU
 * (different streams or host threads without ordering between them) race and
 * give wrong sums.  Calls ordered on one stream are safe.
 * Errors: HEGET_E_INVALID_ARG, HEGET_E_DEVICE. */
heget_status heget_integrate_step_noalloc(heget_process_t p, int64_t n_events, const double* sqrt_s,
                                          const double* uniforms, const int32_t* helicity, double alpha_s,
                                          const heget_cuts* cuts, double* momenta, double* me2, double* weight,
                                          double* sums, void* stream);

/* ---------------------------------------------------------------------------
 * Test hooks (not on the hot path).  They let a test compare the amplitudes
 * themselves, not only |M|^2, with an independent implementation.
 * ------------------------------------------------------------------------- */

/* The reduced colour space the kernels accumulate in.  The kernels never form
 * the K colour-basis amplitudes J of eq. (color-amplitude) explicitly: they add
 * every diagram into y = M J, a vector of K' <= K components (M exact,
 * rational), and evaluate the colour sum of eq. (color-averaged-amplitude) as
 * y^H W y, which equals J^H N J exactly.  The kernels evaluate n_slots helicity
 * configurations per event (leg 0 at helicity +1, structural zeros of massless
 * quark chirality skipped; the all-flipped configurations give the same colour
 * sum and are accounted for by a factor 2).
 *   k_reduced, n_slots  receive K' and the number of evaluated configurations
 *                       (required).
 *   m_num, m_den        HOST int64 [K' * K] or NULL: M = m_num / m_den, row-major.
 *   w_num, w_den        HOST int64 [K' * K'] or NULL: W = w_num / w_den, row-major.
 *   slot_helicity       HOST int32 [n_slots] or NULL: the helicity bit pattern of
 *                       each configuration (bit i set: leg i at +1), in the
 *                       order of the jamp output of heget_matrix_elements_hook.
 * Errors: HEGET_E_INVALID_ARG for a NULL handle, k_reduced or n_slots. */
heget_status heget_colour_reduction(heget_process_t p, int* k_reduced, int* n_slots, int64_t* m_num,
                                    int64_t* m_den, int64_t* w_num, int64_t* w_den, int32_t* slot_helicity);

/* heget_matrix_elements through the test-hook kernels, which are generated
 * from the same diagram graph, routines and colour reduction as the hot-path
 * kernels, for processes with at most six legs, in the handle's precision.
 *   gauge_leg  -1, or the index of a gluon leg whose polarisation vector is
 *              replaced by its momentum divided by its energy (eps -> k/E).
 *              Current conservation (section 4: the three- and four-gluon
 *              vertices of eqs. vvv-amplitude and gggg-amplitude and the qqg
 *              vertex of eq. qqg-amplitude, with the colour factors of
 *              section 2.1) makes every helicity amplitude, and so me2, vanish
 *              up to rounding; a wrong relative sign or colour factor between
 *              diagram types does not.
 *   me2        DEVICE float64 [n_events], written (as heget_matrix_elements).
 *   jamp       DEVICE float64 [n_events][n_slots][K'][2] or NULL: the reduced
 *              colour vector y (real, imaginary part) of every evaluated
 *              configuration, with couplings set to 1: the amplitudes carry
 *              g_s^(n-2) less than eq. (color-amplitude) and phase conventions
 *              of the external states of their own, so y equals
 *              c * M J for one complex c of modulus g_s^-(n-2) per event and
 *              configuration.
 * Other arguments as heget_matrix_elements.
 * Errors: HEGET_E_UNSUPPORTED_PROCESS (no test-hook kernels for this process),
 * HEGET_E_INVALID_ARG (gauge_leg not -1 and not a gluon leg, or as
 * heget_matrix_elements), HEGET_E_DEVICE. */
heget_status heget_matrix_elements_hook(heget_process_t p, const double* momenta, int64_t n_events, double alpha_s,
                                        int gauge_leg, double* me2, double* jamp, void* stream);

/* Release a handle and its device state.  NULL is ignored.  The caller must
 * make sure no queued work still uses the handle.  Cached batch graphs that
 * launch the handle's kernels are destroyed with it. */
void heget_destroy_process(heget_process_t p);

/* Static description of a status code. */
const char* heget_status_string(heget_status s);

/* Processes compiled into the library: their count and normalised specs
 * (index out of range returns NULL). */
int heget_num_processes(void);
const char* heget_process_spec(int index);

#ifdef __cplusplus
}
#endif

#endif /* HEGET_H */
