/*
 * rtcc3.h -- C ABI of the MI355X real-time CC3 library (librtcc3.so).
 *
 * The library propagates the complex closed-shell amplitudes (t1, t2, l1, l2)
 * of real-time CC3 (arXiv 2407.18947) under an electric field in the dipole
 * approximation and returns the induced dipole moment.
 *
 *   Hamiltonian      H(t) = F + U - mu.E(t)                 (Sec. 2.1, eq. cc3-h-pert; Sec. 2.2.1)
 *   amplitude EOMs   i dt/dt = <mu|Hbar|0>, -i dl/dt = dL/dt (eq. cc3-rt-t, eq. cc3-rt-l, Appendix A)
 *   triples          t3 closed form built per occupied triple (i,j,k), divided by the
 *                    orbital-energy denominator, contracted into the singles/doubles
 *                    residuals (eq. cc3-t3-no-pert, cc3-l3, cc3-x1-exp ... cc3-y2-exp; Sec. 2.1)
 *   dipole           mu_x = sum_pq D_pq mu^x_pq with the CC3 one-electron density
 *                    (Sec. 2.2.3; eq. cc3-dij and the two equations after it)
 *   propagation      classic RK4 (Sec. 3)
 *
 * Conventions.  o occupied and v virtual orbitals, n = o + v, occupied first.
 * All arrays are row-major.  Complex numbers are interleaved (re, im) doubles,
 * layout-compatible with std::complex<double> and torch.complex128.
 * State vector y (length 2*(o*v + o*o*v*v)): [ t1[i][a] | t2[i][j][a][b] | l1[i][a] | l2[i][j][a][b] ]
 * with t2[i][j][a][b] = t_ij^ab = t2[j][i][b][a] (same for l2).  The doubles
 * multipliers pair with the residual as 1/2 sum_ijab l2_ijab Omega_ijab, i.e.
 * l2_ijab = <Lambda| E_ai E_bj |0>.
 *
 * Errors.  Every function returns RTCC3_OK (0) or a negative RTCC3_* code;
 * no exception or abort crosses the ABI.  rtcc3_last_error() gives a message.
 * Ownership.  Host arrays passed in are copied; the caller keeps them.  Device
 * pointers passed to rtcc3_rhs / rtcc3_rhs_terms are caller-owned and must stay
 * valid for the call; all work is ordered on the context's stream (the library
 * forks two streams of its own from it and joins them back within each call)
 * and the functions return after that stream has been synchronised.  A
 * context serves one thread at a time.
 * Memory.  rtcc3_create allocates every device buffer the context will use (it
 * evaluates the right-hand side once, on the zero state, to size them); no
 * later call allocates device memory, except rtcc3_set_option with
 * RTCC3_OPT_WINDOW_BLOCKS, which replaces the window buffers, and with
 * RTCC3_OPT_TANGENT, which adds the derivative buffers.  A request that would
 * need more memory after creation fails with RTCC3_ESTATE.
 */
#ifndef RTCC3_H
#define RTCC3_H

#ifdef __cplusplus
extern "C" {
#endif

typedef struct rtcc3_ctx rtcc3_ctx;

typedef struct {
  double re, im;
} rtcc3_c64;

enum {
  RTCC3_OK = 0,
  RTCC3_EINVAL = -1,    /* bad argument (sizes, NULL, non-finite, asymmetric input) */
  RTCC3_ENOMEM = -2,    /* device allocation failed */
  RTCC3_EDEVICE = -3,   /* HIP runtime error (message from hipGetErrorString) */
  RTCC3_ESTATE = -4,    /* call not valid in the context's current state */
  RTCC3_EDIVERGED = -5  /* the propagated state became non-finite */
};

/* Precision of the triples contractions (the paper's single- versus
 * double-precision comparison, Section 3 and Table 1).  Denominators, residual
 * accumulation, RK4 and the dipole always stay in FP64.
 *   RTCC3_FP64    FP64 matrix cores (complex products as three real products)
 *   RTCC3_FP32    operands rounded to FP32, FP32 matrix cores and accumulation
 *   RTCC3_BF16X3  each real operand split into three bf16 slices (about FP32's
 *                 24 significand bits), six slice products on the bf16 matrix
 *                 cores, FP32 accumulation
 *   RTCC3_BF16X2  two bf16 slices (16 bits), three slice products
 * The bf16 splits apply to the segmented products (the builds of t3 and
 * lambda3 and the S intermediate of Y1); the other triples products of such a
 * run use FP32, except the X2 product with an operand combined from three
 * blocks and the 16-wide gathered products, which use FP64 (faster there). */
enum { RTCC3_FP64 = 0, RTCC3_FP32 = 1, RTCC3_BF16X3 = 2, RTCC3_BF16X2 = 3 };

/* Create a context.
 *   o, v     numbers of occupied / virtual orbitals (o >= 1, v >= 1)
 *   fock     [n*n] host, canonical Fock matrix; must be diagonal (|off-diag| <= 1e-12), finite
 *   naux, B  [naux*n*n] host, density-fitting factors, (pq|rs) = sum_P B[P][p][q] B[P][r][s];
 *            each B[P] symmetric (<= 1e-12)
 *   dipole   [3*n*n] host, electric dipole matrices mu^x, mu^y, mu^z, symmetric
 *   precision one of RTCC3_FP64, RTCC3_FP32, RTCC3_BF16X3, RTCC3_BF16X2
 *   hip_stream a hipStream_t to order work on, or NULL for a stream owned by the context
 *   out      receives the context
 * Returns EINVAL, ENOMEM or EDEVICE on failure (message via rtcc3_last_error(NULL)). */
int rtcc3_create(int o, int v, const double *fock, int naux, const double *B, const double *dipole,
                 int precision, void *hip_stream, rtcc3_ctx **out);

/* Set / get the state vector y (layout above).  y_on_device: 0 = host pointer,
 * 1 = device pointer (caller-owned). */
int rtcc3_set_state(rtcc3_ctx *ctx, const rtcc3_c64 *y, int y_on_device);
int rtcc3_get_state(rtcc3_ctx *ctx, rtcc3_c64 *y, int y_on_device);

/* dy = f(y) at field E[3] (host).  y_dev, dy_dev: device arrays of the state length. */
int rtcc3_rhs(rtcc3_ctx *ctx, const double E[3], const rtcc3_c64 *y_dev, rtcc3_c64 *dy_dev);

/* Individual terms of the right-hand side at state y_dev and field E (device
 * output terms_dev, caller-owned), concatenated in this order:
 *   Omega1[o*v]  Omega2[o*o*v*v]     CCSD part of <mu|Hbar|0>
 *   G1[o*v]      G2[o*o*v*v]         CCSD part of dL/dt1, sym(dL/dt2)/(1/2)
 *   X1[o*v]      X2[o*o*v*v]         triples into the T equations (eq. cc3-x1-exp, cc3-x2-exp)
 *   Y1[o*v]      Y2[o*o*v*v]         triples into the Lambda equations (eq. cc3-y1-exp, cc3-y2-exp)
 *   D[n*n]                           one-electron density, T1-transformed frame
 *   mu[3]                            dipole moment
 * with_triples = 0 gives the CCSD model (X, Y and the triples density zero). */
int rtcc3_rhs_terms(rtcc3_ctx *ctx, const double E[3], const rtcc3_c64 *y_dev, rtcc3_c64 *terms_dev,
                    int with_triples);

/* Propagate the context's state by `steps` RK4 steps of size dt (dt != 0).
 *   field       [(2*steps+1)*3] host: E(k*dt/2), k = 0..2*steps
 *   dipole_out  [(steps+1)*3] host: mu(t_n) for n = 0..steps (complex; may be NULL)
 * Each step's new state is checked on the device before it replaces the old
 * one.  If a step gives a non-finite element, the call returns RTCC3_EDIVERGED
 * (its message names the step), the state is left at the last finite state
 * (after the steps before that one), and dipole_out holds the dipoles up to
 * that state and NaN after it.  The dipoles of up to 1024 steps are kept on the
 * device and copied out in chunks. */
int rtcc3_propagate(rtcc3_ctx *ctx, int steps, double dt, const double *field, rtcc3_c64 *dipole_out);

/* Propagate n contexts together, `steps` RK4 steps of size dt each, context i
 * under field fields[i] (layout as rtcc3_propagate) with its dipoles into
 * dipole_out[i] (may be NULL, or NULL entries).  Step s of every context is
 * enqueued on that context's own streams before step s + 1 of any, so the
 * systems (field strengths, directions, systems of different sizes) share the
 * device; each context must have a stream of its own (EINVAL otherwise).
 * Returns the first member's error code (the message, naming the member, via
 * rtcc3_last_error(NULL)); each context is left as rtcc3_propagate leaves it. */
int rtcc3_propagate_batch(rtcc3_ctx *const *ctxs, int n, int steps, double dt, const double *const *fields,
                          rtcc3_c64 *const *dipole_out);

/* Dipole of the context's current state at field E[3] (host) -> out[3] (host). */
int rtcc3_dipole(rtcc3_ctx *ctx, const double E[3], rtcc3_c64 out[3]);

/* Derivatives along a direction (forward mode; RTCC3_OPT_TANGENT first).  The
 * right-hand side f(y, E) is a polynomial in the amplitudes and affine in the
 * field (eq. cc3-rt-t, eq. cc3-rt-l, with h = h0 - mu.E of Sec. 2.2.1), and so
 * is the dipole (Sec. 2.2.3); every kernel of the evaluation has its
 * derivative applied beside it (each product C = A B adds A' B + A B').
 *
 * rtcc3_rhs_tangent: dy = f(y, E) and dydot = (df/dy) ydot + (df/dE) Edot at
 * field E[3] with field direction Edot[3] (host), state y_dev and direction
 * ydot_dev (device, state length, caller-owned; also dy_dev, dydot_dev).
 * mu, mudot (host [3], may be NULL): the dipole at (y, E) and its derivative
 * along the same direction.  The context's state is not changed. */
int rtcc3_rhs_tangent(rtcc3_ctx *ctx, const double E[3], const double Edot[3], const rtcc3_c64 *y_dev,
                      const rtcc3_c64 *ydot_dev, rtcc3_c64 *dy_dev, rtcc3_c64 *dydot_dev, rtcc3_c64 mu[3],
                      rtcc3_c64 mudot[3]);

/* rtcc3_propagate_tangent: `steps` RK4 steps as rtcc3_propagate (same field
 * layout; each step's kernels launched from the host, on the context's
 * stream only), together with the derivative of the dipole series along a
 * direction of the inputs:
 *   field_dot   [(2*steps+1)*3] host: direction of the field samples (may be NULL: zero)
 *   kappa_dot   direction of a scale of the dipole integrals, mu -> (1 + kappa) mu
 *               in both the coupling -mu.E and the dipole, taken at kappa = 0
 *   ydot0       [state length] host: direction of the initial state (may be NULL: zero)
 *   dipole_out, dipole_dot [(steps+1)*3] host: mu(t_n) and d mu(t_n)/ds (may be NULL)
 * The state and its derivative advance together (the derivative of each RK4
 * stage is that of the right-hand side at the stage); rtcc3_get_state_tangent
 * reads the derivative of the final state.  With field_dot = the field's shape
 * at unit amplitude, dipole_dot is the derivative of the dipole series with
 * respect to the field amplitude (at a delta kick of vanishing amplitude, the
 * linear response whose transform gives the polarisability, Sec. 2.2.1 and 2.2.2).
 * Returns RTCC3_EDIVERGED if the state, its derivative or a dipole becomes
 * non-finite (nothing is restored). */
int rtcc3_propagate_tangent(rtcc3_ctx *ctx, int steps, double dt, const double *field, const double *field_dot,
                            double kappa_dot, const rtcc3_c64 *ydot0, rtcc3_c64 *dipole_out,
                            rtcc3_c64 *dipole_dot);

/* Derivative of the context's state after rtcc3_propagate_tangent (zero before
 * any; layout and y_on_device as rtcc3_get_state). */
int rtcc3_get_state_tangent(rtcc3_ctx *ctx, rtcc3_c64 *ydot, int y_on_device);

/* Options: RTCC3_OPT_TRIPLES (1 = CC3, 0 = CCSD model), RTCC3_OPT_PRECISION,
 * RTCC3_OPT_WINDOW_BLOCKS: the most ordered occupied triples (i,j,k) whose t3
 * and lambda3 blocks are held at once (16 * v*v*(2*vp + o) bytes each, vp = v rounded
 * up to a multiple of 8, twice that with RTCC3_OPT_TANGENT); 0 (default)
 * sizes the windows from half the free device memory, at most 48 GiB.  Values
 * below 6 count as 6 (a window holds every ordering of a triple), and the
 * windows of the density pass hold whole slabs (i,l,k) of an occupied pair
 * (l,k), about 6*o blocks, however small the value.  The answer does not
 * depend on it.  Setting it waits for the context's streams, frees the window
 * buffers and allocates those of the new size (the state is kept).
 * RTCC3_OPT_SINGLE_STREAM: 1 = every kernel on the context's stream, one after
 * another (for timing each kernel alone); 0 (default) = the lambda3 side of the
 * triples and the CCSD reverse sweep on two streams of the context's own.  The
 * answer does not depend on it (up to the order of atomic additions).  Setting
 * it waits for the context's streams.
 * RTCC3_OPT_GRAPH: 1 = rtcc3_propagate captures one RK4 step (all its kernels,
 * on all the context's streams) as a HIP graph at its first call with a given
 * dt, precision and stream setting, and replays it for every step (the runtime
 * may allocate for the graph when it is instantiated); 0 (default) = every
 * kernel launched from the host each step.  The answer does not depend on it;
 * with it, rtcc3_last_timing reports the total time only.
 * RTCC3_OPT_AUTOTUNE: the K split of every product whose grid is small enough
 * for it to matter is chosen by timing the feasible splits once, at creation
 * (on the zero state, one stream); 1 = tune again now, 0 = forget the choices
 * (the library's heuristic then).  The answer depends on it only through the
 * order of atomic additions.
 * RTCC3_OPT_TANGENT: 1 = allocate the derivative buffers that rtcc3_rhs_tangent
 * and rtcc3_propagate_tangent need (a twin of every buffer of the context, so
 * as much device memory again); these calls return RTCC3_ESTATE without it.
 * Needs o <= 15 (EINVAL otherwise).  0 is ignored (the buffers stay until
 * rtcc3_destroy). */
enum {
  RTCC3_OPT_TRIPLES = 1,
  RTCC3_OPT_PRECISION = 2,
  RTCC3_OPT_WINDOW_BLOCKS = 3,
  RTCC3_OPT_SINGLE_STREAM = 4,
  RTCC3_OPT_GRAPH = 5,
  RTCC3_OPT_AUTOTUNE = 6,
  RTCC3_OPT_TANGENT = 7
};
int rtcc3_set_option(rtcc3_ctx *ctx, int option, int value);

/* Timing of the last rtcc3_propagate (milliseconds, from HIP events on the
 * context's stream): total and the part spent in the triples kernels.
 * kernel_ms[0] = total, [1] = triples, [2] = triples launches counted,
 * [3] = milliseconds in the segmented products that build t3 and lambda3
 * (eq. cc3-t3 and eq. cc3-l3 before symmetrisation) and the S intermediate of
 * Y1, [4] = their launches, [5] = their algorithmic flops (8 per complex
 * multiply-add). */
int rtcc3_last_timing(rtcc3_ctx *ctx, double kernel_ms[6]);

/* Library self-test of the complex GEMM the contractions run on:
 * C[m][n] = sum_k A[m][k] B[k][n] for host row-major complex arrays, computed
 * on the device with the matrix-core arithmetic of the given precision.
 * Returns EINVAL for non-positive sizes or NULL pointers. */
int rtcc3_zgemm_selftest(int M, int N, int K, int precision, const rtcc3_c64 *A, const rtcc3_c64 *B, rtcc3_c64 *C);

/* The same self-test for callers that cannot allocate device memory (code
 * under HIP graph capture, tight loops, harnesses that forbid hipMalloc): A, B
 * and C are staged in a fixed device array of the library (64 MiB, held by
 * each device the library runs on until the process ends) instead of buffers
 * allocated per call; no hipMalloc, hipFree or allocating library routine is
 * called.  Arguments and results as rtcc3_zgemm_selftest, on the current
 * device.  Returns EINVAL when M*K + K*N + M*N exceeds 4194304 complex
 * elements (message via rtcc3_last_error(NULL)).  All calls on one device
 * share the array: calls that overlap on one device (other threads) race. */
int rtcc3_zgemm_selftest_noalloc(int M, int N, int K, int precision, const rtcc3_c64 *A, const rtcc3_c64 *B,
                                 rtcc3_c64 *C);

/* Autotuner summary: out[0] = products tuned, out[1] = those that run with a
 * K split other than the library's heuristic. */
int rtcc3_tuning_summary(rtcc3_ctx *ctx, int out[2]);

/* The autotuner's choices: up to max_records rows of 8 doubles into out (host),
 * each (M, N, K, batch, heuristic split, chosen split, heuristic ms, chosen ms)
 * of one tuned product; returns the number of tuned products (or EINVAL). */
int rtcc3_tuning_report(rtcc3_ctx *ctx, double *out, int max_records);

const char *rtcc3_last_error(const rtcc3_ctx *ctx); /* ctx == NULL: last create() error of this thread */
void rtcc3_destroy(rtcc3_ctx *ctx);

#ifdef __cplusplus
}
#endif
#endif /* RTCC3_H */
