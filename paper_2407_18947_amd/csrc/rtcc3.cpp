// C ABI of the RT-CC3 library: context, validation, right-hand side, RK4.
#include "../../include/rtcc3.h"

#include <cmath>
#include <cstring>
#include <memory>
#include <string>
#include <vector>

#include "ccsd.h"
#include "engine.h"
#include "triples.h"

using namespace rtcc3;

struct rtcc3_ctx {
  Dims d{};
  hipStream_t stream = nullptr;
  bool own_stream = false;
  std::unique_ptr<Engine> e;
  std::unique_ptr<Triples> tri;
  int precision = RTCC3_FP64;
  int with_triples = 1;
  int64_t ylen = 0;
  View B, mu, h0, I, ones_o, h;
  cplx *y = nullptr, *ytmp = nullptr, *k = nullptr, *acc = nullptr;
  double last_ms[6] = {0, 0, 0, 0, 0, 0};
  cplx* mus = nullptr;      // dipole series of up to kMusSteps steps (+1), copied out per chunk
  cplx* mu_out = nullptr;   // dipole of rtcc3_dipole
  int* pst = nullptr;       // propagation state on the device (PST_*: step, chunk base, divergence flag)
  double* ftab = nullptr;   // field samples E(k dt/2) of the current chunk, 3 doubles each
  double* estage = nullptr; // the four stage fields of the current step
  // one RK4 step captured as a graph (RTCC3_OPT_GRAPH), valid for these settings
  int use_graph = 0;
  Tuner* tuner = nullptr;  // K splits of the products, tuned at set-up
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
  double g_dt = 0.0;
  int g_tri = -1, g_prec = -1, g_single = -1;
  std::string err;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  // the CCSD reverse sweep runs on side_stream beside the triples windows
  // (on stream itself with single_stream)
  hipStream_t side_stream = nullptr;
  int single_stream = 0;
  hipEvent_t ev_side0 = nullptr, ev_res = nullptr, ev_side1 = nullptr;
  // derivative buffers (RTCC3_OPT_TANGENT): the engine's twins, and
  int tangent_ready = 0;
  cplx* zero_nn = nullptr;      // a zero n x n matrix (h0 of the field derivative of h)
  cplx* mu_dot_out = nullptr;   // derivative of the dipole, device [3]
};

namespace {

thread_local std::string g_create_error;

int fail(rtcc3_ctx* c, int code, const std::string& msg) {
  if (c)
    c->err = msg;
  else
    g_create_error = msg;
  return code;
}

template <typename F>
int guarded(rtcc3_ctx* c, F&& f) {
  try {
    return f();
  } catch (const Error& ex) {
    return fail(c, ex.code, ex.what());
  } catch (const std::bad_alloc&) {
    return fail(c, RTCC3_ENOMEM, "host allocation failed");
  } catch (const std::exception& ex) {
    return fail(c, RTCC3_EDEVICE, ex.what());
  }
}

constexpr cplx ONE{1.0, 0.0};
inline cplx C(double re, double im = 0.0) { return cplx{re, im}; }

View sub(cplx* p, int64_t off, std::vector<int64_t> shape) { return Engine::raw(p + off, shape); }

// The field of one right-hand side: three host doubles, or three device doubles
// (the propagation's stage fields, so that a step is the same work every time).
struct FieldRef {
  const double* host = nullptr;
  const double* dev = nullptr;
  const double* dot = nullptr;  // host direction of the field (tangent mode)
};

struct TermsOut {
  cplx* terms = nullptr;    // optional rtcc3_rhs_terms layout
  cplx* mu = nullptr;       // optional dipole (device, 3)
  cplx* mu_dot = nullptr;   // optional derivative of the dipole (device, 3; tangent mode)
  bool mu_at_step = false;  // dipole into the propagation's series at the device step counter
};

// dy = f(y) at field E; optionally the individual terms and/or the dipole.
void rhs_impl(rtcc3_ctx* c, FieldRef E, const cplx* y, cplx* dy, const TermsOut& t, bool with_triples) {
  Engine& e = *c->e;
  const Dims& d = c->d;
  const int64_t o = d.o, v = d.v, n = d.n;
  const int64_t ov = o * v, oovv = o * o * v * v;
  TunerScope tuned(c->tuner);
  // h = h0 - sum_x E_x mu^x
  build_h(c->h.p, c->h0.p, c->mu.p, n * n, E.dev, E.host, c->stream);
  if (e.tangent()) {  // h' = -sum_x Edot_x mu^x
    RTCC3_CHECK(E.dot != nullptr, "tangent: field direction missing");
    build_h(e.twin_out(c->h.p), c->zero_nn, c->mu.p, n * n, nullptr, E.dot, c->stream);
  }
  CCSDResult r = ccsd_forward(e, d, y, c->h, c->B, c->I, c->ones_o);
  // The triples read only the dressed integrals and Fock matrix of the forward
  // part: with more than one stream the residual runs on the side stream,
  // beside the triples' integral blocks (einsums on the two streams use
  // separate scratch), and the reverse sweep follows it there.
  hipEvent_t residual_done = nullptr;
  if (with_triples && !c->single_stream) {
    RTCC3_HIP(hipEventRecord(c->ev_side0, c->stream));
    RTCC3_HIP(hipStreamWaitEvent(c->side_stream, c->ev_side0, 0));
    e.stream = c->side_stream;
    try {
      ccsd_residual(e, d, r);
    } catch (...) {
      e.stream = c->stream;
      throw;
    }
    e.stream = c->stream;
    RTCC3_HIP(hipEventRecord(c->ev_res, c->side_stream));
    residual_done = c->ev_res;
  } else {
    ccsd_residual(e, d, r);
  }
  const bool want_density = t.terms || t.mu || t.mu_at_step;

  TriplesOut to;
  if (with_triples) {
    // the reverse sweep needs only the CCSD forward part and residual: it runs
    // on the side stream after the residual, beside the triples work
    to = c->tri->run(e, d, r, y, want_density, [&](hipEvent_t after) -> hipEvent_t {
      // With bf16 slices the builds are not bound by the matrix cores and the
      // sweep starts as soon as the residual is done, beside them; with FP64
      // or FP32 products it waits for the lambda3 build, so that the builds
      // share the chip only with the memory-bound symmetrisation.
      const bool early = !c->single_stream && (c->precision == RTCC3_BF16X3 || c->precision == RTCC3_BF16X2);
      if (!early) RTCC3_HIP(hipStreamWaitEvent(c->side_stream, after, 0));
      e.stream = c->single_stream ? c->stream : c->side_stream;
      try {
        ccsd_backward(e, d, y, c->ones_o, r);
      } catch (...) {
        e.stream = c->stream;
        throw;
      }
      e.stream = c->stream;
      RTCC3_HIP(hipEventRecord(c->ev_side1, c->side_stream));
      return c->ev_side1;
    }, residual_done);
    // the reverse sweep's gradients are read below
    if (hipEvent_t sd = c->tri->side_done()) RTCC3_HIP(hipStreamWaitEvent(c->stream, sd, 0));
  } else {
    ccsd_backward(e, d, y, c->ones_o, r);
  }

  if (dy) {
    e.zero(Engine::raw(dy, {c->ylen}));
    View dt1 = sub(dy, 0, {o, v}), dt2 = sub(dy, ov, {o, o, v, v});
    View dl1 = sub(dy, ov + oovv, {o, v}), dl2 = sub(dy, 2 * ov + oovv, {o, o, v, v});
    e.axpy(C(0, -1), r.R1, dt1);
    e.axpy(C(0, -1), r.R2, dt2);
    e.axpy(C(0, 1), r.G1, dl1);
    // -i dl2/dt = sym(dL/dt2) / (1/2) = G2 + G2^T(ij,ab)
    e.axpy(C(0, 1), r.G2, dl2);
    e.axpy(C(0, 1), Engine::permute(r.G2, {1, 0, 3, 2}), dl2);
    if (with_triples) {
      e.axpy(C(0, -1), to.X1, dt1);
      e.axpy(C(0, -1), to.X2, dt2);
      e.axpy(C(0, 1), to.Y1, dl1);
      e.axpy(C(0, 1), to.Y2, dl2);
    }
  }

  if (want_density) {
    // D = D_ccsd + triples terms (T1-transformed frame); mu_x = sum_pq D_pq mu~^x_pq
    View D = e.tensor("Dtot", {n, n});
    e.zero(D);
    e.axpy(ONE, r.Dt, D);
    if (with_triples) {
      e.axpy(ONE, to.Dij, Engine::slice(Engine::slice(D, 0, 0, o), 1, 0, o));
      e.axpy(ONE, to.Dab, Engine::slice(Engine::slice(D, 0, o, n), 1, o, n));
      e.axpy(ONE, to.Dia, Engine::slice(Engine::slice(D, 0, 0, o), 1, o, n));
    }
    View muX = e.tensor("muX", {3, n, n});
    e.zero(muX);
    e.einsum("pr,xrs->xps", ONE, r.X, c->mu, muX);
    View mut = e.tensor("mut", {3, n, n});
    e.zero(mut);
    e.einsum("xps,sq->xpq", ONE, muX, r.Y, mut);
    View m3 = e.tensor("mu3", {3});
    e.zero(m3);
    e.einsum("pq,xpq->x", ONE, D, mut, m3);
    if (t.mu) copy(t.mu, m3.p, 3, c->stream);
    if (t.mu_dot) {
      const cplx* m3t = e.twin(m3.p);
      if (m3t)
        copy(t.mu_dot, m3t, 3, c->stream);
      else
        fill(t.mu_dot, 3, cplx{0, 0}, c->stream);
    }
    if (t.mu_at_step) store_dipole(c->mus, m3.p, c->pst, c->stream);
    if (t.terms) {
      cplx* p = t.terms;
      auto put = [&](const View& src, int64_t len) {
        if (src.p)
          RTCC3_HIP(hipMemcpyAsync(p, src.p, sizeof(cplx) * len, hipMemcpyDeviceToDevice, c->stream));
        else
          fill(p, len, cplx{0, 0}, c->stream);
        p += len;
      };
      put(r.R1, ov);
      put(r.R2, oovv);
      put(r.G1, ov);
      // G2 reported symmetrised: G2 + G2^T
      {
        View g = sub(p, 0, {o, o, v, v});
        fill(p, oovv, cplx{0, 0}, c->stream);
        e.axpy(ONE, r.G2, g);
        e.axpy(ONE, Engine::permute(r.G2, {1, 0, 3, 2}), g);
        p += oovv;
      }
      put(with_triples ? to.X1 : View(), ov);
      put(with_triples ? to.X2 : View(), oovv);
      put(with_triples ? to.Y1 : View(), ov);
      put(with_triples ? to.Y2 : View(), oovv);
      put(D, n * n);
      put(m3, 3);
    }
  }
}

// Steps whose dipoles are held on the device before they are copied out.
constexpr int kMusSteps = 1024;

// Evaluate the right-hand side once for every kind of pass (the density pass
// with the dipole, the plain right-hand side) on the current state, so that
// every buffer, scratch area and gradient the evaluation uses is allocated
// now; then seal the engine, after which a propagation allocates nothing.
void warm_up(rtcc3_ctx* c, bool tune) {
  static const double E0[3] = {0.0, 0.0, 0.0};
  c->e->seal(false);
  TermsOut t;
  t.mu = c->mu_out;
  if (tune) {
    // the K splits are timed one product at a time, all on one stream; repeating
    // a product is harmless here, where every result is discarded
    const int single = c->single_stream;
    c->single_stream = 1;
    c->tri->set_single_stream(true);
    tuner_set_tuning(c->tuner, true);
    try {
      rhs_impl(c, FieldRef{E0, nullptr}, c->y, c->k, t, true);
      rhs_impl(c, FieldRef{E0, nullptr}, c->y, c->k, TermsOut{}, true);
    } catch (...) {
      tuner_set_tuning(c->tuner, false);
      c->single_stream = single;
      c->tri->set_single_stream(single != 0);
      throw;
    }
    tuner_set_tuning(c->tuner, false);
    c->single_stream = single;
    c->tri->set_single_stream(single != 0);
  }
  rhs_impl(c, FieldRef{E0, nullptr}, c->y, c->k, t, true);
  rhs_impl(c, FieldRef{E0, nullptr}, c->y, c->k, TermsOut{}, true);
  RTCC3_HIP(hipStreamSynchronize(c->stream));
  RTCC3_HIP(hipStreamSynchronize(c->side_stream));
  c->tri->reset_timing();
  c->e->seal(true);
}

void drop_graph(rtcc3_ctx* c) {
  if (c->gexec) (void)hipGraphExecDestroy(c->gexec);
  if (c->graph) (void)hipGraphDestroy(c->graph);
  c->gexec = nullptr;
  c->graph = nullptr;
}

// One RK4 step of the context's state, the same work every step: the stage
// fields come from the device field table at the device step counter, the
// dipole of the step's starting state goes to the counter's slot of the
// series, and the counter advances at the end, so a captured graph of it can
// be replayed step after step.
void step_body(rtcc3_ctx* c, double dt, bool tri) {
  Engine& e = *c->e;
  const int64_t L = c->ylen;
  View YT = Engine::raw(c->ytmp, {L}), K = Engine::raw(c->k, {L}), A = Engine::raw(c->acc, {L});
  auto copyL = [&](cplx* dst, const cplx* src) { copy(dst, src, L, c->stream); };
  stage_fields(c->ftab, c->pst, c->estage, c->stream);
  TermsOut t;
  t.mu_at_step = true;
  rhs_impl(c, FieldRef{nullptr, c->estage}, c->y, c->k, t, tri);  // k1 (and mu(t_s))
  copyL(c->acc, c->k);
  copyL(c->ytmp, c->y);
  e.axpy(C(0.5 * dt), K, YT);
  rhs_impl(c, FieldRef{nullptr, c->estage + 3}, c->ytmp, c->k, TermsOut{}, tri);  // k2
  e.axpy(C(2.0), K, A);
  copyL(c->ytmp, c->y);
  e.axpy(C(0.5 * dt), K, YT);
  rhs_impl(c, FieldRef{nullptr, c->estage + 6}, c->ytmp, c->k, TermsOut{}, tri);  // k3
  e.axpy(C(2.0), K, A);
  copyL(c->ytmp, c->y);
  e.axpy(C(dt), K, YT);
  rhs_impl(c, FieldRef{nullptr, c->estage + 9}, c->ytmp, c->k, TermsOut{}, tri);  // k4
  e.axpy(ONE, K, A);
  // y += dt/6 (k1 + 2 k2 + 2 k3 + k4) unless the result is not finite: then y
  // keeps its last finite value (ytmp is free after k4)
  guarded_update(c->y, c->acc, C(dt / 6.0), c->ytmp, L, c->pst, c->stream);
  advance_step(c->pst, c->stream);
}

// The step captured as a graph, once per step size and settings.
void ensure_graph(rtcc3_ctx* c, double dt, bool tri) {
  if (c->gexec && c->g_dt == dt && c->g_tri == (int)tri && c->g_prec == c->precision &&
      c->g_single == c->single_stream)
    return;
  drop_graph(c);
  c->tri->set_timing(false);
  RTCC3_HIP(hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
  try {
    step_body(c, dt, tri);
  } catch (...) {
    hipGraph_t g = nullptr;
    (void)hipStreamEndCapture(c->stream, &g);
    if (g) (void)hipGraphDestroy(g);
    c->tri->set_timing(true);
    throw;
  }
  hipGraph_t g = nullptr;
  const hipError_t ec = hipStreamEndCapture(c->stream, &g);
  c->tri->set_timing(true);
  RTCC3_HIP(ec);
  c->graph = g;
  RTCC3_HIP(hipGraphInstantiate(&c->gexec, c->graph, nullptr, nullptr, 0));
  c->g_dt = dt;
  c->g_tri = (int)tri;
  c->g_prec = c->precision;
  c->g_single = c->single_stream;
}

// The propagation of one context: fields and dipoles in chunks of kMusSteps
// steps, each step eager or a replay of the captured graph.
struct Runner {
  rtcc3_ctx* c;
  int steps;
  double dt;
  const double* field;
  bool tri;
  std::vector<cplx> mh;
  int base = 0;

  void chunk(int s0) {  // the fields of the steps from s0 on, counter reset to s0
    const int n = std::min(kMusSteps, steps - s0);
    RTCC3_HIP(hipMemcpyAsync(c->ftab, field + 6 * (size_t)s0, sizeof(double) * 3 * (2 * (size_t)n + 1),
                             hipMemcpyHostToDevice, c->stream));
    reset_step(c->pst, s0, c->stream);
    base = s0;
  }
  void flush(int upto) {  // dipoles base .. upto - 1 to the host (waits for them)
    RTCC3_HIP(hipMemcpyAsync(mh.data() + 3 * (size_t)base, c->mus, sizeof(cplx) * 3 * (size_t)(upto - base),
                             hipMemcpyDeviceToHost, c->stream));
    RTCC3_HIP(hipStreamSynchronize(c->stream));
  }
  void begin() {
    mh.assign((size_t)(steps + 1) * 3, cplx{0, 0});
    c->tri->reset_timing();
    if (c->use_graph && steps > 0) ensure_graph(c, dt, tri);
    fill_int(c->pst, PST_N, 0, c->stream);
    RTCC3_HIP(hipEventRecord(c->ev0, c->stream));
  }
  void step(int s) {
    if (s % kMusSteps == 0) {
      if (s > 0) flush(s);
      chunk(s);
    }
    if (c->use_graph)
      RTCC3_HIP(hipGraphLaunch(c->gexec, c->stream));
    else
      step_body(c, dt, tri);
  }
  int finish(rtcc3_c64* dipole_out) {
    if (steps == 0) {
      chunk(0);
    } else if (steps - base == kMusSteps) {
      flush(steps);
      chunk(steps);
    }
    stage_fields(c->ftab, c->pst, c->estage, c->stream);
    TermsOut t;
    t.mu_at_step = true;
    rhs_impl(c, FieldRef{nullptr, c->estage}, c->y, nullptr, t, tri);
    RTCC3_HIP(hipEventRecord(c->ev1, c->stream));
    int ph[PST_N] = {0, 0, 0, 0};
    RTCC3_HIP(hipMemcpyAsync(ph, c->pst, sizeof(ph), hipMemcpyDeviceToHost, c->stream));
    flush(steps + 1);
    float ms = 0.f;
    RTCC3_HIP(hipEventElapsedTime(&ms, c->ev0, c->ev1));
    c->last_ms[0] = ms;
    c->tri->fold_timing();
    c->tri->timing(c->last_ms[1], c->last_ms[2]);
    c->tri->build_timing(c->last_ms[3], c->last_ms[4], c->last_ms[5]);
    const int bad = ph[PST_FLAG];
    if (bad) {
      // step bad - 1 gave a non-finite state: y is the state after bad - 1 steps,
      // whose dipoles (indices 0 .. bad - 1) are valid; the later ones are not
      const double nan = std::nan("");
      for (size_t q = (size_t)bad; q < (size_t)steps + 1; ++q)
        mh[3 * q] = mh[3 * q + 1] = mh[3 * q + 2] = cplx{nan, nan};
    }
    if (dipole_out) std::memcpy(dipole_out, mh.data(), sizeof(cplx) * mh.size());
    if (bad)
      return fail(c, RTCC3_EDIVERGED,
                  "state became non-finite in step " + std::to_string(bad - 1) + "; the state is left after " +
                      std::to_string(bad - 1) + " steps");
    for (auto& z : mh)
      if (!std::isfinite(z.re) || !std::isfinite(z.im)) return fail(c, RTCC3_EDIVERGED, "dipole became non-finite");
    return RTCC3_OK;
  }
};

// Tangent mode for one call: every kernel on the context's stream (the
// derivative launches follow their products in order), restored afterwards.
struct TangentScope {
  rtcc3_ctx* c;
  int single;
  explicit TangentScope(rtcc3_ctx* cc) : c(cc), single(cc->single_stream) {
    c->single_stream = 1;
    c->tri->set_single_stream(true);
    c->e->set_tangent(true);
  }
  ~TangentScope() {
    c->e->set_tangent(false);
    c->single_stream = single;
    c->tri->set_single_stream(single != 0);
  }
};

bool finite(const double* p, int64_t n) {
  for (int64_t i = 0; i < n; ++i)
    if (!std::isfinite(p[i])) return false;
  return true;
}

}  // namespace

void rtcc3::set_thread_error(const std::string& msg) { g_create_error = msg; }

// =============================================================================

static_assert(RTCC3_FP64 == RTCC3_PREC_FP64 && RTCC3_FP32 == RTCC3_PREC_FP32 && RTCC3_BF16X3 == RTCC3_PREC_BF16X3 &&
                  RTCC3_BF16X2 == RTCC3_PREC_BF16X2,
              "precision codes of the C interface and the kernels differ");

extern "C" int rtcc3_create(int o, int v, const double* fock, int naux, const double* B, const double* dipole,
                            int precision, void* hip_stream, rtcc3_ctx** out) {
  if (!out) return fail(nullptr, RTCC3_EINVAL, "out is NULL");
  *out = nullptr;
  if (o < 1 || v < 1) return fail(nullptr, RTCC3_EINVAL, "need o >= 1 and v >= 1");
  if (naux < 1) return fail(nullptr, RTCC3_EINVAL, "need naux >= 1");
  if (!fock || !B || !dipole) return fail(nullptr, RTCC3_EINVAL, "NULL input array");
  if (precision < RTCC3_FP64 || precision > RTCC3_BF16X2) return fail(nullptr, RTCC3_EINVAL, "unknown precision");
  const int64_t n = (int64_t)o + v;
  if (n > 4096 || (int64_t)naux * n * n > (int64_t)1 << 34)
    return fail(nullptr, RTCC3_ENOMEM, "system too large");
  if (!finite(fock, n * n) || !finite(B, (int64_t)naux * n * n) || !finite(dipole, 3 * n * n))
    return fail(nullptr, RTCC3_EINVAL, "non-finite input");
  for (int64_t p = 0; p < n; ++p)
    for (int64_t q = 0; q < n; ++q)
      if (p != q && std::fabs(fock[p * n + q]) > 1e-12) return fail(nullptr, RTCC3_EINVAL, "Fock matrix is not diagonal");
  for (int64_t P = 0; P < naux; ++P)
    for (int64_t p = 0; p < n; ++p)
      for (int64_t q = 0; q < p; ++q)
        if (std::fabs(B[(P * n + p) * n + q] - B[(P * n + q) * n + p]) > 1e-12)
          return fail(nullptr, RTCC3_EINVAL, "B[P] is not symmetric");
  for (int x = 0; x < 3; ++x)
    for (int64_t p = 0; p < n; ++p)
      for (int64_t q = 0; q < p; ++q)
        if (std::fabs(dipole[(x * n + p) * n + q] - dipole[(x * n + q) * n + p]) > 1e-12)
          return fail(nullptr, RTCC3_EINVAL, "dipole matrix is not symmetric");
  for (int64_t p = 0; p < o; ++p)
    for (int64_t a = o; a < n; ++a)
      if (!(fock[p * n + p] < fock[a * n + a]))
        return fail(nullptr, RTCC3_EINVAL, "occupied orbital energies must lie below the virtual ones");

  std::unique_ptr<rtcc3_ctx> c(new rtcc3_ctx());
  int rc = guarded(nullptr, [&]() -> int {
    c->d = Dims{o, v, (int)n, naux};
    c->precision = precision;
    if (hip_stream) {
      c->stream = (hipStream_t)hip_stream;
    } else {
      RTCC3_HIP(hipStreamCreate(&c->stream));
      c->own_stream = true;
    }
    RTCC3_HIP(hipEventCreate(&c->ev0));
    RTCC3_HIP(hipEventCreate(&c->ev1));
    RTCC3_HIP(hipStreamCreateWithFlags(&c->side_stream, hipStreamNonBlocking));
    RTCC3_HIP(hipEventCreateWithFlags(&c->ev_side0, hipEventDisableTiming));
    RTCC3_HIP(hipEventCreateWithFlags(&c->ev_res, hipEventDisableTiming));
    RTCC3_HIP(hipEventCreateWithFlags(&c->ev_side1, hipEventDisableTiming));
    c->e.reset(new Engine(c->stream));
    Engine& e = *c->e;
    // constants in complex form
    std::vector<cplx> hb((size_t)naux * n * n);
    for (size_t i = 0; i < hb.size(); ++i) hb[i] = cplx{B[i], 0.0};
    c->B = e.tensor("B", {naux, n, n});
    RTCC3_HIP(hipMemcpyAsync(c->B.p, hb.data(), sizeof(cplx) * hb.size(), hipMemcpyHostToDevice, c->stream));
    std::vector<cplx> hm((size_t)3 * n * n);
    for (size_t i = 0; i < hm.size(); ++i) hm[i] = cplx{dipole[i], 0.0};
    c->mu = e.tensor("mu", {3, n, n});
    RTCC3_HIP(hipMemcpyAsync(c->mu.p, hm.data(), sizeof(cplx) * hm.size(), hipMemcpyHostToDevice, c->stream));
    // h0 = f - sum_i [2 (pq|ii) - (pi|iq)] so that the reference Fock matrix is f
    std::vector<double> J((size_t)n * n, 0.0), K((size_t)n * n, 0.0), bd(naux, 0.0);
    for (int64_t P = 0; P < naux; ++P)
      for (int64_t i = 0; i < o; ++i) bd[P] += B[(P * n + i) * n + i];
    for (int64_t P = 0; P < naux; ++P) {
      const double* b = B + P * n * n;
      for (int64_t p = 0; p < n; ++p)
        for (int64_t q = 0; q < n; ++q) {
          J[p * n + q] += b[p * n + q] * bd[P];
          double s = 0.0;
          for (int64_t i = 0; i < o; ++i) s += b[p * n + i] * b[i * n + q];
          K[p * n + q] += s;
        }
    }
    std::vector<cplx> h0((size_t)n * n);
    for (int64_t p = 0; p < n; ++p)
      for (int64_t q = 0; q < n; ++q)
        h0[p * n + q] = cplx{(p == q ? fock[p * n + p] : 0.0) - (2.0 * J[p * n + q] - K[p * n + q]), 0.0};
    c->h0 = e.tensor("h0", {n, n});
    RTCC3_HIP(hipMemcpyAsync(c->h0.p, h0.data(), sizeof(cplx) * h0.size(), hipMemcpyHostToDevice, c->stream));
    c->h = e.tensor("h", {n, n});
    std::vector<cplx> eye((size_t)n * n, cplx{0, 0});
    for (int64_t p = 0; p < n; ++p) eye[p * n + p] = cplx{1, 0};
    c->I = e.tensor("I", {n, n});
    RTCC3_HIP(hipMemcpyAsync(c->I.p, eye.data(), sizeof(cplx) * eye.size(), hipMemcpyHostToDevice, c->stream));
    std::vector<cplx> ones(o, cplx{1, 0});
    c->ones_o = e.tensor("ones_o", {o});
    RTCC3_HIP(hipMemcpyAsync(c->ones_o.p, ones.data(), sizeof(cplx) * o, hipMemcpyHostToDevice, c->stream));
    std::vector<double> eps(n);
    for (int64_t p = 0; p < n; ++p) eps[p] = fock[p * n + p];
    c->tri.reset(new Triples(e, c->d, eps, precision));
    c->ylen = 2 * ((int64_t)o * v + (int64_t)o * o * v * v);
    c->y = e.tensor("y", {c->ylen}).p;
    c->ytmp = e.tensor("ytmp", {c->ylen}).p;
    c->k = e.tensor("k", {c->ylen}).p;
    c->acc = e.tensor("acc", {c->ylen}).p;
    c->mus = e.tensor("mus", {kMusSteps + 1, 3}).p;
    c->mu_out = e.tensor("mu_out", {3}).p;
    c->pst = (int*)e.tensor("pst", {(PST_N * (int64_t)sizeof(int) + 15) / 16}).p;
    c->ftab = (double*)e.tensor("ftab", {(3 * (2 * (int64_t)kMusSteps + 1) + 1) / 2}).p;
    c->estage = (double*)e.tensor("estage", {6}).p;
    // every buffer of an evaluation now, none while propagating (the state is
    // zero), and the K splits of the products
    c->tuner = tuner_new();
    warm_up(c.get(), true);
    return RTCC3_OK;
  });
  if (rc != RTCC3_OK) {
    g_create_error = c->err.empty() ? g_create_error : c->err;
    return rc;
  }
  *out = c.release();
  return RTCC3_OK;
}

extern "C" int rtcc3_set_state(rtcc3_ctx* c, const rtcc3_c64* y, int y_on_device) {
  if (!c) return RTCC3_EINVAL;
  if (!y) return fail(c, RTCC3_EINVAL, "y is NULL");
  return guarded(c, [&]() -> int {
    if (!y_on_device) {
      const double* p = (const double*)y;
      if (!finite(p, 2 * c->ylen)) return fail(c, RTCC3_EINVAL, "non-finite state");
    }
    RTCC3_HIP(hipMemcpyAsync(c->y, y, sizeof(cplx) * c->ylen, y_on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice,
                             c->stream));
    RTCC3_HIP(hipStreamSynchronize(c->stream));
    return RTCC3_OK;
  });
}

extern "C" int rtcc3_get_state(rtcc3_ctx* c, rtcc3_c64* y, int y_on_device) {
  if (!c) return RTCC3_EINVAL;
  if (!y) return fail(c, RTCC3_EINVAL, "y is NULL");
  return guarded(c, [&]() -> int {
    RTCC3_HIP(hipMemcpyAsync(y, c->y, sizeof(cplx) * c->ylen, y_on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost,
                             c->stream));
    RTCC3_HIP(hipStreamSynchronize(c->stream));
    return RTCC3_OK;
  });
}

static bool field_ok(const double* E) { return E && std::isfinite(E[0]) && std::isfinite(E[1]) && std::isfinite(E[2]); }

extern "C" int rtcc3_rhs(rtcc3_ctx* c, const double E[3], const rtcc3_c64* y_dev, rtcc3_c64* dy_dev) {
  if (!c) return RTCC3_EINVAL;
  if (!field_ok(E)) return fail(c, RTCC3_EINVAL, "field must be 3 finite numbers");
  if (!y_dev || !dy_dev) return fail(c, RTCC3_EINVAL, "NULL state pointer");
  return guarded(c, [&]() -> int {
    rhs_impl(c, FieldRef{E, nullptr}, (const cplx*)y_dev, (cplx*)dy_dev, TermsOut{}, c->with_triples != 0);
    RTCC3_HIP(hipStreamSynchronize(c->stream));
    c->tri->fold_timing();
    return RTCC3_OK;
  });
}

extern "C" int rtcc3_rhs_terms(rtcc3_ctx* c, const double E[3], const rtcc3_c64* y_dev, rtcc3_c64* terms_dev,
                               int with_triples) {
  if (!c) return RTCC3_EINVAL;
  if (!field_ok(E)) return fail(c, RTCC3_EINVAL, "field must be 3 finite numbers");
  if (!y_dev || !terms_dev) return fail(c, RTCC3_EINVAL, "NULL pointer");
  return guarded(c, [&]() -> int {
    TermsOut t;
    t.terms = (cplx*)terms_dev;
    rhs_impl(c, FieldRef{E, nullptr}, (const cplx*)y_dev, nullptr, t, with_triples != 0);
    RTCC3_HIP(hipStreamSynchronize(c->stream));
    c->tri->fold_timing();
    return RTCC3_OK;
  });
}

extern "C" int rtcc3_dipole(rtcc3_ctx* c, const double E[3], rtcc3_c64 out[3]) {
  if (!c) return RTCC3_EINVAL;
  if (!field_ok(E) || !out) return fail(c, RTCC3_EINVAL, "bad argument");
  return guarded(c, [&]() -> int {
    TermsOut t;
    t.mu = c->mu_out;
    rhs_impl(c, FieldRef{E, nullptr}, c->y, nullptr, t, c->with_triples != 0);
    RTCC3_HIP(hipMemcpyAsync(out, c->mu_out, sizeof(cplx) * 3, hipMemcpyDeviceToHost, c->stream));
    RTCC3_HIP(hipStreamSynchronize(c->stream));
    c->tri->fold_timing();
    return RTCC3_OK;
  });
}

namespace {

int check_propagate_args(rtcc3_ctx* c, int steps, double dt, const double* field) {
  if (steps < 0) return fail(c, RTCC3_EINVAL, "steps < 0");
  if (!(std::isfinite(dt)) || dt == 0.0) return fail(c, RTCC3_EINVAL, "dt must be finite and non-zero");
  if (!field) return fail(c, RTCC3_EINVAL, "field is NULL");
  if (!finite(field, (int64_t)(2 * steps + 1) * 3)) return fail(c, RTCC3_EINVAL, "non-finite field");
  return RTCC3_OK;
}

}  // namespace

extern "C" int rtcc3_propagate(rtcc3_ctx* c, int steps, double dt, const double* field, rtcc3_c64* dipole_out) {
  if (!c) return RTCC3_EINVAL;
  if (int rc = check_propagate_args(c, steps, dt, field)) return rc;
  return guarded(c, [&]() -> int {
    Runner r{c, steps, dt, field, c->with_triples != 0};
    r.begin();
    for (int s = 0; s < steps; ++s) r.step(s);
    return r.finish(dipole_out);
  });
}

extern "C" int rtcc3_propagate_batch(rtcc3_ctx* const* ctxs, int n, int steps, double dt, const double* const* fields,
                                     rtcc3_c64* const* dipole_out) {
  if (!ctxs || n < 1) return fail(nullptr, RTCC3_EINVAL, "batch: need at least one context");
  if (!fields) return fail(nullptr, RTCC3_EINVAL, "batch: fields is NULL");
  for (int i = 0; i < n; ++i) {
    if (!ctxs[i]) return fail(nullptr, RTCC3_EINVAL, "batch: NULL context");
    for (int j = 0; j < i; ++j)
      if (ctxs[j] == ctxs[i] || ctxs[j]->stream == ctxs[i]->stream)
        return fail(nullptr, RTCC3_EINVAL, "batch: contexts must be distinct and on distinct streams");
    if (int rc = check_propagate_args(ctxs[i], steps, dt, fields[i])) {
      set_thread_error(ctxs[i]->err);
      return rc;
    }
  }
  std::vector<Runner> rs;
  int rc = guarded(ctxs[0], [&]() -> int {
    for (int i = 0; i < n; ++i) rs.push_back(Runner{ctxs[i], steps, dt, fields[i], ctxs[i]->with_triples != 0});
    for (auto& r : rs) r.begin();
    // lockstep: step s of every context is enqueued on its own streams before step s + 1
    for (int s = 0; s < steps; ++s)
      for (auto& r : rs) r.step(s);
    int first = RTCC3_OK;
    for (int i = 0; i < n; ++i) {
      const int ri = rs[i].finish(dipole_out ? dipole_out[i] : nullptr);
      if (ri != RTCC3_OK && first == RTCC3_OK) {
        first = ri;
        set_thread_error("batch member " + std::to_string(i) + ": " + ctxs[i]->err);
      }
    }
    return first;
  });
  if (rc != RTCC3_OK && rc != RTCC3_EDIVERGED) set_thread_error(ctxs[0]->err);
  return rc;
}

extern "C" int rtcc3_rhs_tangent(rtcc3_ctx* c, const double E[3], const double Edot[3], const rtcc3_c64* y_dev,
                                 const rtcc3_c64* ydot_dev, rtcc3_c64* dy_dev, rtcc3_c64* dydot_dev, rtcc3_c64 mu[3],
                                 rtcc3_c64 mudot[3]) {
  if (!c) return RTCC3_EINVAL;
  if (!c->tangent_ready) return fail(c, RTCC3_ESTATE, "derivative buffers not allocated (RTCC3_OPT_TANGENT)");
  if (!field_ok(E) || !field_ok(Edot)) return fail(c, RTCC3_EINVAL, "field and its direction must be 3 finite numbers");
  if (!y_dev || !ydot_dev || !dy_dev || !dydot_dev) return fail(c, RTCC3_EINVAL, "NULL state pointer");
  return guarded(c, [&]() -> int {
    Engine& e = *c->e;
    const int64_t L = c->ylen;
    TangentScope ts(c);
    // the state and its direction into the context's stage buffer and its twin
    RTCC3_HIP(hipMemcpyAsync(c->ytmp, y_dev, sizeof(cplx) * L, hipMemcpyDeviceToDevice, c->stream));
    RTCC3_HIP(hipMemcpyAsync(e.twin_out(c->ytmp), ydot_dev, sizeof(cplx) * L, hipMemcpyDeviceToDevice, c->stream));
    TermsOut t;
    t.mu = c->mu_out;
    t.mu_dot = c->mu_dot_out;
    rhs_impl(c, FieldRef{E, nullptr, Edot}, c->ytmp, c->k, t, c->with_triples != 0);
    RTCC3_HIP(hipMemcpyAsync(dy_dev, c->k, sizeof(cplx) * L, hipMemcpyDeviceToDevice, c->stream));
    const cplx* kt = e.twin(c->k);
    if (kt)
      RTCC3_HIP(hipMemcpyAsync(dydot_dev, kt, sizeof(cplx) * L, hipMemcpyDeviceToDevice, c->stream));
    else
      RTCC3_HIP(hipMemsetAsync(dydot_dev, 0, sizeof(cplx) * L, c->stream));
    if (mu) RTCC3_HIP(hipMemcpyAsync(mu, c->mu_out, sizeof(cplx) * 3, hipMemcpyDeviceToHost, c->stream));
    if (mudot) RTCC3_HIP(hipMemcpyAsync(mudot, c->mu_dot_out, sizeof(cplx) * 3, hipMemcpyDeviceToHost, c->stream));
    RTCC3_HIP(hipStreamSynchronize(c->stream));
    c->tri->fold_timing();
    return RTCC3_OK;
  });
}

extern "C" int rtcc3_propagate_tangent(rtcc3_ctx* c, int steps, double dt, const double* field,
                                       const double* field_dot, double kappa_dot, const rtcc3_c64* ydot0,
                                       rtcc3_c64* dipole_out, rtcc3_c64* dipole_dot) {
  if (!c) return RTCC3_EINVAL;
  if (!c->tangent_ready) return fail(c, RTCC3_ESTATE, "derivative buffers not allocated (RTCC3_OPT_TANGENT)");
  if (int rc = check_propagate_args(c, steps, dt, field)) return rc;
  const int64_t nf = (int64_t)(2 * steps + 1) * 3;
  if (field_dot && !finite(field_dot, nf)) return fail(c, RTCC3_EINVAL, "non-finite field direction");
  if (!std::isfinite(kappa_dot)) return fail(c, RTCC3_EINVAL, "non-finite kappa_dot");
  if (ydot0 && !finite((const double*)ydot0, 2 * c->ylen)) return fail(c, RTCC3_EINVAL, "non-finite state direction");
  return guarded(c, [&]() -> int {
    Engine& e = *c->e;
    const int64_t L = c->ylen;
    const bool tri = c->with_triples != 0;
    TangentScope ts(c);
    cplx* yt = e.twin_out(c->y);
    if (ydot0)
      RTCC3_HIP(hipMemcpyAsync(yt, ydot0, sizeof(cplx) * L, hipMemcpyHostToDevice, c->stream));
    else
      fill(yt, L, cplx{0, 0}, c->stream);
    // the direction of the field that h sees: d/ds of (1 + kappa) E at kappa = 0
    std::vector<double> fd((size_t)nf);
    for (int64_t q = 0; q < nf; ++q) fd[q] = (field_dot ? field_dot[q] : 0.0) + kappa_dot * field[q];
    std::vector<cplx> mh((size_t)(steps + 1) * 3), mdh((size_t)(steps + 1) * 3);
    View YT = Engine::raw(c->ytmp, {L}), K = Engine::raw(c->k, {L}), A = Engine::raw(c->acc, {L}),
         Y = Engine::raw(c->y, {L});
    auto sample = [&](int k) { return FieldRef{field + 3 * (size_t)k, nullptr, fd.data() + 3 * (size_t)k}; };
    auto dipoles = [&](int step) {
      RTCC3_HIP(hipMemcpyAsync(mh.data() + 3 * (size_t)step, c->mu_out, sizeof(cplx) * 3, hipMemcpyDeviceToHost,
                               c->stream));
      RTCC3_HIP(hipMemcpyAsync(mdh.data() + 3 * (size_t)step, c->mu_dot_out, sizeof(cplx) * 3,
                               hipMemcpyDeviceToHost, c->stream));
    };
    TermsOut t;
    t.mu = c->mu_out;
    t.mu_dot = c->mu_dot_out;
    RTCC3_HIP(hipEventRecord(c->ev0, c->stream));
    for (int n = 0; n < steps; ++n) {
      rhs_impl(c, sample(2 * n), c->y, c->k, t, tri);  // k1 (and mu(t_n))
      dipoles(n);
      e.copy(c->acc, c->k, L);
      e.copy(c->ytmp, c->y, L);
      e.axpy(C(0.5 * dt), K, YT);
      rhs_impl(c, sample(2 * n + 1), c->ytmp, c->k, TermsOut{}, tri);  // k2
      e.axpy(C(2.0), K, A);
      e.copy(c->ytmp, c->y, L);
      e.axpy(C(0.5 * dt), K, YT);
      rhs_impl(c, sample(2 * n + 1), c->ytmp, c->k, TermsOut{}, tri);  // k3
      e.axpy(C(2.0), K, A);
      e.copy(c->ytmp, c->y, L);
      e.axpy(C(dt), K, YT);
      rhs_impl(c, sample(2 * n + 2), c->ytmp, c->k, TermsOut{}, tri);  // k4
      e.axpy(ONE, K, A);
      e.axpy(C(dt / 6.0), A, Y);
    }
    rhs_impl(c, sample(2 * steps), c->y, nullptr, t, tri);
    dipoles(steps);
    RTCC3_HIP(hipEventRecord(c->ev1, c->stream));
    RTCC3_HIP(hipStreamSynchronize(c->stream));
    float ms = 0.f;
    RTCC3_HIP(hipEventElapsedTime(&ms, c->ev0, c->ev1));
    c->last_ms[0] = ms;
    c->tri->fold_timing();
    c->tri->timing(c->last_ms[1], c->last_ms[2]);
    c->tri->build_timing(c->last_ms[3], c->last_ms[4], c->last_ms[5]);
    // the dipole operator itself scales with 1 + kappa
    for (size_t q = 0; q < mh.size(); ++q) {
      mdh[q].re += kappa_dot * mh[q].re;
      mdh[q].im += kappa_dot * mh[q].im;
    }
    if (dipole_out) std::memcpy(dipole_out, mh.data(), sizeof(cplx) * mh.size());
    if (dipole_dot) std::memcpy(dipole_dot, mdh.data(), sizeof(cplx) * mdh.size());
    for (size_t q = 0; q < mh.size(); ++q)
      if (!std::isfinite(mh[q].re) || !std::isfinite(mh[q].im) || !std::isfinite(mdh[q].re) ||
          !std::isfinite(mdh[q].im))
        return fail(c, RTCC3_EDIVERGED, "dipole or its derivative became non-finite");
    return RTCC3_OK;
  });
}

extern "C" int rtcc3_get_state_tangent(rtcc3_ctx* c, rtcc3_c64* ydot, int y_on_device) {
  if (!c) return RTCC3_EINVAL;
  if (!ydot) return fail(c, RTCC3_EINVAL, "ydot is NULL");
  if (!c->tangent_ready) return fail(c, RTCC3_ESTATE, "derivative buffers not allocated (RTCC3_OPT_TANGENT)");
  return guarded(c, [&]() -> int {
    const cplx* yt = c->e->twin(c->y);
    const hipMemcpyKind kind = y_on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
    if (yt) {
      RTCC3_HIP(hipMemcpyAsync(ydot, yt, sizeof(cplx) * c->ylen, kind, c->stream));
    } else if (y_on_device) {
      RTCC3_HIP(hipMemsetAsync(ydot, 0, sizeof(cplx) * c->ylen, c->stream));
    } else {
      std::memset(ydot, 0, sizeof(cplx) * c->ylen);
    }
    RTCC3_HIP(hipStreamSynchronize(c->stream));
    return RTCC3_OK;
  });
}

extern "C" int rtcc3_set_option(rtcc3_ctx* c, int option, int value) {
  if (!c) return RTCC3_EINVAL;
  if (option == RTCC3_OPT_TRIPLES) {
    c->with_triples = value ? 1 : 0;
    return RTCC3_OK;
  }
  if (option == RTCC3_OPT_AUTOTUNE) {
    return guarded(c, [&]() -> int {
      RTCC3_HIP(hipStreamSynchronize(c->side_stream));
      drop_graph(c);  // captured with the old splits
      tuner_clear(c->tuner);
      if (!value) return RTCC3_OK;
      std::vector<cplx> keep((size_t)c->ylen);
      RTCC3_HIP(hipMemcpy(keep.data(), c->y, sizeof(cplx) * keep.size(), hipMemcpyDeviceToHost));
      fill(c->y, c->ylen, cplx{0, 0}, c->stream);
      warm_up(c, true);
      RTCC3_HIP(hipMemcpy(c->y, keep.data(), sizeof(cplx) * keep.size(), hipMemcpyHostToDevice));
      return RTCC3_OK;
    });
  }
  if (option == RTCC3_OPT_GRAPH) {
    c->use_graph = value ? 1 : 0;
    if (!c->use_graph) drop_graph(c);
    return RTCC3_OK;
  }
  if (option == RTCC3_OPT_PRECISION) {
    if (value < RTCC3_FP64 || value > RTCC3_BF16X2) return fail(c, RTCC3_EINVAL, "unknown precision");
    c->precision = value;
    c->tri->set_precision(value);
    return RTCC3_OK;
  }
  if (option == RTCC3_OPT_SINGLE_STREAM) {
    return guarded(c, [&]() -> int {
      RTCC3_HIP(hipStreamSynchronize(c->stream));
      RTCC3_HIP(hipStreamSynchronize(c->side_stream));
      c->single_stream = value ? 1 : 0;
      c->tri->set_single_stream(value != 0);
      return RTCC3_OK;
    });
  }
  if (option == RTCC3_OPT_TANGENT) {
    if (!value || c->tangent_ready) return RTCC3_OK;
    if (c->d.o > 15) return fail(c, RTCC3_EINVAL, "derivatives need o <= 15");
    return guarded(c, [&]() -> int {
      RTCC3_HIP(hipStreamSynchronize(c->side_stream));
      drop_graph(c);
      Engine& e = *c->e;
      e.seal(false);
      const int64_t n = c->d.n;
      c->zero_nn = e.tensor("zero_nn", {n, n}).p;
      c->mu_dot_out = e.tensor("mu_dot_out", {3}).p;
      e.enable_twins();
      // one derivative evaluation of each kind on the zero state and direction,
      // so that nothing is allocated later
      static const double E0[3] = {0.0, 0.0, 0.0};
      std::vector<cplx> keep((size_t)c->ylen);
      RTCC3_HIP(hipMemcpy(keep.data(), c->y, sizeof(cplx) * keep.size(), hipMemcpyDeviceToHost));
      fill(c->y, c->ylen, cplx{0, 0}, c->stream);
      {
        TangentScope ts(c);
        TermsOut t;
        t.mu = c->mu_out;
        t.mu_dot = c->mu_dot_out;
        rhs_impl(c, FieldRef{E0, nullptr, E0}, c->y, c->k, t, true);
        rhs_impl(c, FieldRef{E0, nullptr, E0}, c->y, c->k, TermsOut{}, true);
      }
      RTCC3_HIP(hipStreamSynchronize(c->stream));
      RTCC3_HIP(hipMemcpy(c->y, keep.data(), sizeof(cplx) * keep.size(), hipMemcpyHostToDevice));
      c->tri->reset_timing();
      e.seal(true);
      c->tangent_ready = 1;
      return RTCC3_OK;
    });
  }
  if (option == RTCC3_OPT_WINDOW_BLOCKS) {
    if (value < 0) return fail(c, RTCC3_EINVAL, "negative window size");
    return guarded(c, [&]() -> int {
      RTCC3_HIP(hipStreamSynchronize(c->side_stream));
      drop_graph(c);  // it refers to the window buffers being replaced
      c->e->seal(false);
      c->tri->set_window_blocks(*c->e, value);
      // the window buffers of the new size now, none later; the state is kept
      std::vector<cplx> keep((size_t)c->ylen);
      RTCC3_HIP(hipMemcpy(keep.data(), c->y, sizeof(cplx) * keep.size(), hipMemcpyDeviceToHost));
      fill(c->y, c->ylen, cplx{0, 0}, c->stream);
      warm_up(c, false);
      RTCC3_HIP(hipMemcpy(c->y, keep.data(), sizeof(cplx) * keep.size(), hipMemcpyHostToDevice));
      return RTCC3_OK;
    });
  }
  return fail(c, RTCC3_EINVAL, "unknown option");
}

extern "C" int rtcc3_last_timing(rtcc3_ctx* c, double kernel_ms[6]) {
  if (!c || !kernel_ms) return RTCC3_EINVAL;
  for (int i = 0; i < 6; ++i) kernel_ms[i] = c->last_ms[i];
  return RTCC3_OK;
}

extern "C" int rtcc3_tuning_summary(rtcc3_ctx* c, int out[2]) {
  if (!c || !out) return RTCC3_EINVAL;
  tuner_counts(c->tuner, out[0], out[1]);
  return RTCC3_OK;
}

extern "C" int rtcc3_tuning_report(rtcc3_ctx* c, double* out, int max_records) {
  if (!c || max_records < 0 || (max_records > 0 && !out)) return RTCC3_EINVAL;
  std::vector<TuneRecord> r((size_t)max_records);
  const int n = tuner_records(c->tuner, r.data(), max_records);
  for (int i = 0; i < std::min(n, max_records); ++i) {
    const TuneRecord& t = r[i];
    const double row[8] = {(double)t.M, (double)t.N, (double)t.K, (double)t.batch, (double)t.heuristic,
                           (double)t.chosen, (double)t.heuristic_ms, (double)t.chosen_ms};
    std::memcpy(out + 8 * i, row, sizeof(row));
  }
  return n;
}

extern "C" const char* rtcc3_last_error(const rtcc3_ctx* c) { return c ? c->err.c_str() : g_create_error.c_str(); }

extern "C" void rtcc3_destroy(rtcc3_ctx* c) {
  if (!c) return;
  (void)hipStreamSynchronize(c->stream);
  drop_graph(c);
  c->tri.reset();
  tuner_delete(c->tuner);
  c->e.reset();
  if (c->ev0) (void)hipEventDestroy(c->ev0);
  if (c->ev1) (void)hipEventDestroy(c->ev1);
  if (c->side_stream) (void)hipStreamSynchronize(c->side_stream);
  if (c->ev_side0) (void)hipEventDestroy(c->ev_side0);
  if (c->ev_res) (void)hipEventDestroy(c->ev_res);
  if (c->ev_side1) (void)hipEventDestroy(c->ev_side1);
  if (c->side_stream) (void)hipStreamDestroy(c->side_stream);
  if (c->own_stream) (void)hipStreamDestroy(c->stream);
  delete c;
}

extern "C" int rtcc3_zgemm_selftest(int M, int N, int K, int precision, const rtcc3_c64* A, const rtcc3_c64* B,
                                    rtcc3_c64* Cout) {
  if (M < 1 || N < 1 || K < 1 || !A || !B || !Cout) return fail(nullptr, RTCC3_EINVAL, "bad gemm arguments");
  if (precision < RTCC3_FP64 || precision > RTCC3_BF16X2) return fail(nullptr, RTCC3_EINVAL, "unknown precision");
  if ((int64_t)M * K > (1LL << 28) || (int64_t)K * N > (1LL << 28) || (int64_t)M * N > (1LL << 28))
    return fail(nullptr, RTCC3_EINVAL, "gemm self-test too large");
  cplx *dA = nullptr, *dB = nullptr, *dC = nullptr;
  int rc = guarded(nullptr, [&]() -> int {
    RTCC3_HIP(hipMalloc(&dA, sizeof(cplx) * M * K));
    RTCC3_HIP(hipMalloc(&dB, sizeof(cplx) * K * N));
    RTCC3_HIP(hipMalloc(&dC, sizeof(cplx) * M * N));
    RTCC3_HIP(hipMemcpy(dA, A, sizeof(cplx) * M * K, hipMemcpyHostToDevice));
    RTCC3_HIP(hipMemcpy(dB, B, sizeof(cplx) * K * N, hipMemcpyHostToDevice));
    RTCC3_HIP(hipMemset(dC, 0, sizeof(cplx) * M * N));
    GemmDesc g;
    std::memset(&g, 0, sizeof(g));
    g.M = M;
    g.N = N;
    g.K = K;
    g.M0 = M;
    g.N0 = N;
    g.K0 = K;
    g.batch = 1;
    g.A = dA;
    g.sAm0 = K;
    g.sAk0 = 1;
    g.B = dB;
    g.sBk0 = N;
    g.sBn0 = 1;
    g.C = dC;
    g.sCm0 = N;
    g.sCn0 = 1;
    g.alpha = cplx{1, 0};
    g.prec = precision;
    g.force_prec = 1;
    gemm(g, nullptr);
    RTCC3_HIP(hipDeviceSynchronize());
    RTCC3_HIP(hipMemcpy(Cout, dC, sizeof(cplx) * M * N, hipMemcpyDeviceToHost));
    return RTCC3_OK;
  });
  if (dA) (void)hipFree(dA);
  if (dB) (void)hipFree(dB);
  if (dC) (void)hipFree(dC);
  return rc;
}
