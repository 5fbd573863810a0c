// Triples engine: for windows of ordered occupied triples (i,j,k), build the
// [v,v,v] blocks
//   t_ijk   = P_ijk^abc { sum_e t_ij^ae <cb|ke>~ - sum_m t_im^ab <mc|jk>~ } / D_ijk^abc
//                                         (eq. cc3-t3-no-pert, spin-adapted form in App. A)
//   lambda_ijk = P_ijk^abc { ... } / D_ijk^abc   (eq. cc3-l3-exp with the denominator of eq. cc3-l3)
// on the matrix cores, keep them only for the window, and contract them into
// X1, X2 (eq. cc3-x1-exp, cc3-x2-exp), Y1, Y2 (eq. cc3-y1-exp, cc3-y2-exp) and,
// on request, the density terms (eq. cc3-dij and the two after it).
//
// Y1 uses intermediates accumulated over all blocks and contracted once at the
// end (the factorisation strategy of Sec. 4.1).  The sixth t3.lambda2 term is
// taken with L_kjab and the tenth with <di|lb>, the readings under which the
// printed Y1 equals the derivative of the Lagrangian.
#include "triples.h"

#include <algorithm>
#include <array>
#include <cstring>
#include <map>
#include <tuple>

#include "triples_kernels.h"

namespace rtcc3 {

namespace {

constexpr cplx ONE{1.0, 0.0};
// Timing event pools (pairs); a full pool is folded, which waits for the device.
constexpr int kRunEvents = 512, kBuildEvents = 2048;
inline cplx R(double x) { return cplx{x, 0.0}; }

GemmDesc base(int M, int N, int K, int nb, const int* bl, int prec) {
  GemmDesc g;
  std::memset(&g, 0, sizeof(g));
  g.M = M;
  g.N = N;
  g.K = K;
  g.M0 = M;
  g.N0 = N;
  g.K0 = K;
  g.batch = nb;
  g.bl = bl;
  g.alpha = ONE;
  g.prec = prec;
  return g;
}

// Upper bound of the element offset reached by an index of extent X split as
// (X/X0, X0) with strides (s1, s0).
int64_t span(int64_t X, int64_t X0, int64_t s1, int64_t s0) {
  if (X <= 0) return 0;
  RTCC3_CHECK(s1 >= 0 && s0 >= 0, "triples: negative stride");
  RTCC3_CHECK(X % X0 == 0, "triples: split does not divide the extent");
  return (X / X0 - 1) * s1 + (X0 - 1) * s0;
}

// Launch a GEMM after checking, on the host, that every batch entry stays
// inside the operand buffers (lengths in elements).
void checked_gemm(const GemmDesc& g, const int* bl_host, int64_t lenA, int64_t lenB, int64_t lenC, hipStream_t s) {
  if (g.batch <= 0) return;
  const int64_t eA = span(g.M, g.M0, g.sAm1, g.sAm0) + span(g.K, g.K0, g.sAk1, g.sAk0);
  const int64_t eB = span(g.K, g.K0, g.sBk1, g.sBk0) + span(g.N, g.N0, g.sBn1, g.sBn0);
  const int64_t eC = span(g.M, g.M0, g.sCm1, g.sCm0) + span(g.N, g.N0, g.sCn1, g.sCn0);
  for (int b = 0; b < g.batch; ++b) {
    int64_t oA, oB, oC;
    if (g.bl) {
      const int* q = bl_host + 4 * b;
      oA = g.cA[0] * q[0] + g.cA[1] * q[1] + g.cA[2] * q[2] + g.cA[3] * q[3];
      oB = g.cB[0] * q[0] + g.cB[1] * q[1] + g.cB[2] * q[2] + g.cB[3] * q[3];
      oC = g.cC[0] * q[0] + g.cC[1] * q[1] + g.cC[2] * q[2] + g.cC[3] * q[3];
    } else {
      oA = b * g.sAb;
      oB = b * g.sBb;
      oC = b * g.sCb;
    }
    RTCC3_CHECK(oA >= 0 && oA + eA < lenA, "triples: A operand out of bounds");
    RTCC3_CHECK(oB >= 0 && oB + eB < lenB, "triples: B operand out of bounds");
    RTCC3_CHECK(oC >= 0 && oC + eC < lenC, "triples: C operand out of bounds");
  }
  gemm(g, s);
}

// A gathered-K product (GemmDesc::gk_*) over one grouping of a window's
// contraction blocks after the same check for every gathered block and every
// group's output.
void checked_gather_gemm(GemmDesc& g, const Groups& gr, int64_t lenA, int64_t lenB, int64_t lenC, hipStream_t s) {
  const int ng = (int)gr.key.size() / 4;
  if (ng == 0) return;
  g.batch = ng;
  g.bl = gr.d_key;
  g.gk_start = gr.d_start;
  g.gk_bl = gr.d_bl;
  RTCC3_CHECK(g.K == g.K0 * gr.max && g.sAk1 == 0 && g.sBk1 == 0, "triples: bad gathered product");
  const int64_t eA = span(g.M, g.M0, g.sAm1, g.sAm0) + (int64_t)(g.K0 - 1) * g.sAk0;
  const int64_t eB = (int64_t)(g.K0 - 1) * g.sBk0 + span(g.N, g.N0, g.sBn1, g.sBn0);
  const int64_t eC = span(g.M, g.M0, g.sCm1, g.sCm0) + span(g.N, g.N0, g.sCn1, g.sCn0);
  auto dot = [](const int64_t* c, const int* q) { return c[0] * q[0] + c[1] * q[1] + c[2] * q[2] + c[3] * q[3]; };
  for (int b = 0; b < ng; ++b) {
    const int64_t oC = dot(g.cC, &gr.key[4 * b]);
    RTCC3_CHECK(oC >= 0 && oC + eC < lenC, "triples: C operand out of bounds");
    for (int p = gr.start[b]; p < gr.start[b + 1]; ++p) {
      const int64_t oA = dot(g.cA, &gr.bl[4 * p]), oB = dot(g.cB, &gr.bl[4 * p]);
      RTCC3_CHECK(oA >= 0 && oA + eA < lenA, "triples: A operand out of bounds");
      RTCC3_CHECK(oB >= 0 && oB + eB < lenB, "triples: B operand out of bounds");
    }
  }
  gemm(g, s);
}

// A K-segmented product (GemmDesc::seg) after the same check per segment;
// lenA[s], lenB[s]: lengths of segment s's operand tensors.
void checked_seg_gemm(const GemmDesc& g, const int* bl_host, const int64_t* lenA, const int64_t* lenB, int64_t lenC,
                      hipStream_t s) {
  if (g.batch <= 0) return;
  RTCC3_CHECK(g.bl && g.nseg >= 1 && g.nseg <= 4, "triples: segmented product needs a block table");
  const int64_t eC = span(g.M, g.M0, g.sCm1, g.sCm0) + span(g.N, g.N0, g.sCn1, g.sCn0);
  for (int b = 0; b < g.batch; ++b) {
    const int* q = bl_host + 4 * b;
    const int64_t oC = g.cC[0] * q[0] + g.cC[1] * q[1] + g.cC[2] * q[2] + g.cC[3] * q[3];
    RTCC3_CHECK(oC >= 0 && oC + eC < lenC, "triples: C operand out of bounds");
    for (int t = 0; t < g.nseg; ++t) {
      const GemmDesc::Seg& sg = g.seg[t];
      const int len = sg.len;
      RTCC3_CHECK(len >= 1 && sg.sAm >= 0 && sg.sAk >= 0 && sg.sBk >= 0 && sg.sBn >= 0, "triples: bad segment");
      const int64_t oA = sg.cA[0] * q[0] + sg.cA[1] * q[1] + sg.cA[2] * q[2] + sg.cA[3] * q[3];
      const int64_t oB = sg.cB[0] * q[0] + sg.cB[1] * q[1] + sg.cB[2] * q[2] + sg.cB[3] * q[3];
      const int64_t eA = (int64_t)(g.M - 1) * sg.sAm + (int64_t)(len - 1) * sg.sAk;
      const int64_t eB = (int64_t)(len - 1) * sg.sBk + (int64_t)(g.N - 1) * sg.sBn;
      RTCC3_CHECK(oA >= 0 && oA + eA < lenA[t], "triples: A segment out of bounds");
      RTCC3_CHECK(oB >= 0 && oB + eB < lenB[t], "triples: B segment out of bounds");
    }
  }
  gemm(g, s);
}

// A column-segment product (GemmDesc::cs) after the same check per segment;
// lenB[s], lenC[s]: lengths of segment s's B and C tensors, lenB[4 + s],
// lenC[4 + s] those of its tail column's (when it has one).
void checked_colseg_gemm(const GemmDesc& g, const int* bl_host, int64_t lenA, const int64_t* lenB, const int64_t* lenC,
                         hipStream_t s) {
  if (g.batch <= 0) return;
  RTCC3_CHECK(g.bl && g.ncs >= 1 && g.ncs <= 4, "triples: column segments need a block table");
  const int64_t eA = span(g.M, g.M0, g.sAm1, g.sAm0) + span(g.K, g.K0, g.sAk1, g.sAk0);
  auto dot = [](const int64_t* c, const int* q) { return c[0] * q[0] + c[1] * q[1] + c[2] * q[2] + c[3] * q[3]; };
  for (int b = 0; b < g.batch; ++b) {
    const int* q = bl_host + 4 * b;
    const int64_t oA = dot(g.cA, q);
    RTCC3_CHECK(oA >= 0 && oA + eA < lenA, "triples: A operand out of bounds");
    for (int t = 0; t < g.ncs; ++t) {
      const GemmDesc::ColSeg& c = g.cs[t];
      const int64_t oB = dot(c.cB, q), oC = dot(c.cC, q);
      RTCC3_CHECK(oB >= 0 && oB + (int64_t)(g.K - 1) * c.sBk + (int64_t)(c.n - 1) * c.sBn < lenB[t],
                  "triples: B segment out of bounds");
      RTCC3_CHECK(oC >= 0 && oC + (int64_t)(g.M - 1) * c.sCm + (int64_t)(c.n - 1) * c.sCn < lenC[t],
                  "triples: C segment out of bounds");
      if (c.tB) {
        const int64_t tB = dot(c.tcB, q), tC = dot(c.tcC, q);
        RTCC3_CHECK(tB >= 0 && tB + (int64_t)(g.K - 1) * c.tsBk < lenB[4 + t], "triples: tail B out of bounds");
        RTCC3_CHECK(tC >= 0 && tC + (int64_t)(g.M - 1) * c.tsCm < lenC[4 + t], "triples: tail C out of bounds");
      }
    }
  }
  gemm(g, s);
}

// ---------------------------------------------------------------------------
// Derivatives of the products (tangent mode of the engine): a product
// C (+)= alpha A B adds alpha (A' B + A B') to C', with the twins of the
// operands and of C from the engine.  An operand whose twin is zero adds no
// launch.  A store-mode product stores its first derivative launch and
// accumulates the others; if every twin is zero it clears C' instead.
// ---------------------------------------------------------------------------

void tangent_gemm(Engine& e, const GemmDesc& g, const int* bl_host, int64_t lenA, int64_t lenB, int64_t lenC,
                  hipStream_t s) {
  const cplx* at = e.twin(g.A);
  const cplx* bt = e.twin(g.B);
  RTCC3_CHECK(!g.store, "triples: derivative of a plain store-mode product");
  if (!at && !bt) return;
  cplx* ct = e.twin_out(g.C);
  for (int q = 0; q < 2; ++q) {
    const cplx* x = q == 0 ? at : bt;
    if (!x) continue;
    GemmDesc h = g;
    (q == 0 ? h.A : h.B) = x;
    h.C = ct;
    checked_gemm(h, bl_host, lenA, lenB, lenC, s);
  }
}

void tangent_gather(Engine& e, const GemmDesc& g, const Groups& gr, int64_t lenA, int64_t lenB, int64_t lenC,
                    hipStream_t s) {
  const cplx* at = e.twin(g.A);
  const cplx* bt = e.twin(g.B);
  if (!at && !bt) return;
  cplx* ct = e.twin_out(g.C);
  for (int q = 0; q < 2; ++q) {
    const cplx* x = q == 0 ? at : bt;
    if (!x) continue;
    GemmDesc h = g;
    (q == 0 ? h.A : h.B) = x;
    h.C = ct;
    checked_gather_gemm(h, gr, lenA, lenB, lenC, s);
  }
}

void tangent_seg(Engine& e, const GemmDesc& g, const int* bl_host, const int64_t* lenA, const int64_t* lenB,
                 int64_t lenC, hipStream_t s) {
  struct Term {
    GemmDesc::Seg sg;
    int64_t la, lb;
  };
  std::vector<Term> terms;
  for (int t = 0; t < g.nseg; ++t) {
    const cplx* at = e.twin(g.seg[t].A);
    const cplx* bt = e.twin(g.seg[t].B);
    if (at) {
      terms.push_back(Term{g.seg[t], lenA[t], lenB[t]});
      terms.back().sg.A = at;
    }
    if (bt) {
      terms.push_back(Term{g.seg[t], lenA[t], lenB[t]});
      terms.back().sg.B = bt;
    }
  }
  cplx* ct = e.twin_out(g.C);
  if (terms.empty()) {
    if (g.store) fill(ct, lenC, cplx{0, 0}, s);
    return;
  }
  for (size_t p0 = 0; p0 < terms.size(); p0 += 4) {
    GemmDesc h = g;
    h.C = ct;
    h.nseg = (int)std::min<size_t>(4, terms.size() - p0);
    int64_t la[4], lb[4];
    int k0 = 0;
    for (int q = 0; q < h.nseg; ++q) {
      h.seg[q] = terms[p0 + q].sg;
      h.seg[q].k0 = k0;  // segments start at multiples of 16
      la[q] = terms[p0 + q].la;
      lb[q] = terms[p0 + q].lb;
      if (q + 1 < h.nseg) k0 += (h.seg[q].len + 15) / 16 * 16;
    }
    h.K = h.K0 = k0 + h.seg[h.nseg - 1].len;
    if (p0 > 0 || !g.store) {
      h.store = 0;
      h.atomic = 1;
    }
    checked_seg_gemm(h, bl_host, la, lb, lenC, s);
  }
}

void tangent_colseg(Engine& e, const GemmDesc& g, const int* bl_host, int64_t lenA, const int64_t* lenB,
                    const int64_t* lenC, hipStream_t s) {
  const cplx* at = e.twin(g.A);
  if (at) {  // A' with every segment's B (and tail)
    GemmDesc h = g;
    h.A = at;
    for (int t = 0; t < g.ncs; ++t) {
      h.cs[t].C = e.twin_out(g.cs[t].C);
      if (g.cs[t].tB) h.cs[t].tC = e.twin_out(g.cs[t].tC);
    }
    checked_colseg_gemm(h, bl_host, lenA, lenB, lenC, s);
  }
  // A with the segments' B' (and tails'); a segment whose B' is zero but whose
  // tail's is not runs with a zero scale
  GemmDesc h = g;
  int64_t lb[8] = {0}, lc[8] = {0};
  int ns = 0;
  for (int t = 0; t < g.ncs; ++t) {
    const GemmDesc::ColSeg& c = g.cs[t];
    const cplx* bt = e.twin(c.B);
    const cplx* tbt = c.tB ? e.twin(c.tB) : nullptr;
    if (!bt && !tbt) continue;
    GemmDesc::ColSeg q = c;
    if (bt)
      q.B = bt;
    else
      q.alpha = cplx{0, 0};
    q.C = e.twin_out(c.C);
    if (c.tB) {
      if (tbt)
        q.tB = tbt;
      else
        q.talpha = cplx{0, 0};
      q.tC = e.twin_out(c.tC);
    }
    h.cs[ns] = q;
    lb[ns] = lenB[t];
    lc[ns] = lenC[t];
    lb[4 + ns] = lenB[4 + t];
    lc[4 + ns] = lenC[4 + t];
    ++ns;
  }
  if (ns == 0) return;
  h.ncs = ns;
  h.N = h.N0 = 16 * ns;
  checked_colseg_gemm(h, bl_host, lenA, lb, lc, s);
}

// The products with their derivatives in tangent mode.
void prod(Engine& e, const GemmDesc& g, const int* bl_host, int64_t lenA, int64_t lenB, int64_t lenC, hipStream_t s) {
  checked_gemm(g, bl_host, lenA, lenB, lenC, s);
  if (e.tangent()) tangent_gemm(e, g, bl_host, lenA, lenB, lenC, s);
}
void prod_gather(Engine& e, GemmDesc& g, const Groups& gr, int64_t lenA, int64_t lenB, int64_t lenC, hipStream_t s) {
  checked_gather_gemm(g, gr, lenA, lenB, lenC, s);
  if (e.tangent()) tangent_gather(e, g, gr, lenA, lenB, lenC, s);
}
void prod_seg(Engine& e, const GemmDesc& g, const int* bl_host, const int64_t* lenA, const int64_t* lenB,
              int64_t lenC, hipStream_t s) {
  checked_seg_gemm(g, bl_host, lenA, lenB, lenC, s);
  if (e.tangent()) tangent_seg(e, g, bl_host, lenA, lenB, lenC, s);
}
void prod_colseg(Engine& e, const GemmDesc& g, const int* bl_host, int64_t lenA, const int64_t* lenB,
                 const int64_t* lenC, hipStream_t s) {
  checked_colseg_gemm(g, bl_host, lenA, lenB, lenC, s);
  if (e.tangent()) tangent_colseg(e, g, bl_host, lenA, lenB, lenC, s);
}

// The innermost index of a window block padded to a multiple of 8.
int pad8(int v) { return (v + 7) / 8 * 8; }

void set4(int64_t* c, int64_t a, int64_t b, int64_t d, int64_t n) {
  c[0] = a;
  c[1] = b;
  c[2] = d;
  c[3] = n;
}

}  // namespace

Triples::Triples(Engine& e, const Dims& d, const std::vector<double>& eps, int precision) : d_(d), prec_(precision) {
  RTCC3_HIP(hipMalloc(&eps_, sizeof(double) * eps.size()));
  RTCC3_HIP(hipMemcpy(eps_, eps.data(), sizeof(double) * eps.size(), hipMemcpyHostToDevice));
  build_windows();
  for (auto& w : rhs_windows_) upload(w);
  for (auto& w : den_windows_) upload(w);
  RTCC3_HIP(hipStreamCreateWithFlags(&s2_, hipStreamNonBlocking));
  RTCC3_HIP(hipEventCreateWithFlags(&ev_fork_, hipEventDisableTiming));
  RTCC3_HIP(hipEventCreateWithFlags(&ev_l_, hipEventDisableTiming));
  RTCC3_HIP(hipEventCreateWithFlags(&ev_join_, hipEventDisableTiming));
  RTCC3_HIP(hipEventCreateWithFlags(&ev_t3b_, hipEventDisableTiming));
  RTCC3_HIP(hipEventCreateWithFlags(&ev_t_, hipEventDisableTiming));
  RTCC3_HIP(hipEventCreateWithFlags(&ev_l3b_, hipEventDisableTiming));
  rev_.resize(kRunEvents);
  bev_.resize(kBuildEvents);
  for (auto* pool : {&rev_, &bev_})
    for (hipEvent_t& ev : *pool) RTCC3_HIP(hipEventCreate(&ev));
  (void)e;
}

void Triples::fold_timing() {
  for (int i = 0; i + 1 < nrev_; i += 2) {
    RTCC3_HIP(hipEventSynchronize(rev_[i + 1]));
    float ms = 0;
    RTCC3_HIP(hipEventElapsedTime(&ms, rev_[i], rev_[i + 1]));
    ms_ += ms;
  }
  for (int i = 0; i + 1 < nbev_; i += 2) {
    RTCC3_HIP(hipEventSynchronize(bev_[i + 1]));
    float b = 0;
    RTCC3_HIP(hipEventElapsedTime(&b, bev_[i], bev_[i + 1]));
    build_ms_ += b;
    ++build_launches_;
  }
  nrev_ = nbev_ = 0;
}

void Triples::free_windows() {
  for (auto* ws : {&rhs_windows_, &den_windows_}) {
    for (auto& w : *ws) {
      for (int* p : {w.d_bl, w.d_part, w.d_owned, w.d_canon, w.d_slabs, w.d_orb, w.d_orb_owned, w.d_bk_t3,
                     w.d_bk_l3, w.d_bk_own})
        if (p) (void)hipFree(p);
      for (Groups* gr : {&w.gJ, &w.gK})
        for (int* p : {gr->d_key, gr->d_start, gr->d_bl})
          if (p) (void)hipFree(p);
    }
    ws->clear();
  }
}

void Triples::set_window_blocks(Engine& e, int n) {
  RTCC3_CHECK(n >= 0, "triples: negative window size");
  RTCC3_HIP(hipStreamSynchronize(e.stream));
  RTCC3_HIP(hipStreamSynchronize(s2_));
  free_windows();
  for (const char* b : {"tw_T", "tw_L", "tw_S"}) e.release(b);
  wcap_ = n;
  build_windows();
  for (auto& w : rhs_windows_) upload(w);
  for (auto& w : den_windows_) upload(w);
}

Triples::~Triples() {
  if (s2_) (void)hipStreamSynchronize(s2_);
  free_windows();
  if (eps_) (void)hipFree(eps_);
  for (hipEvent_t ev : {ev_fork_, ev_l_, ev_join_, ev_t3b_, ev_t_, ev_l3b_})
    if (ev) (void)hipEventDestroy(ev);
  if (s2_) (void)hipStreamDestroy(s2_);
  for (hipEvent_t ev : rev_) (void)hipEventDestroy(ev);
  for (hipEvent_t ev : bev_) (void)hipEventDestroy(ev);
}

namespace {

std::vector<std::array<int, 3>> orderings(int x, int y, int z) {
  std::array<int, 3> t{x, y, z};
  std::sort(t.begin(), t.end());
  std::vector<std::array<int, 3>> out;
  do out.push_back(t);
  while (std::next_permutation(t.begin(), t.end()));
  return out;
}

void finish_window(Window& w, const std::vector<std::array<int, 3>>& blocks) {
  std::map<std::array<int, 3>, int> idx;
  for (int n = 0; n < (int)blocks.size(); ++n) idx[blocks[n]] = n;
  w.nw = (int)blocks.size();
  w.bl.resize(4 * w.nw);
  w.part.resize(6 * w.nw);
  for (int n = 0; n < w.nw; ++n) {
    const int I = blocks[n][0], J = blocks[n][1], K = blocks[n][2];
    w.bl[4 * n] = I;
    w.bl[4 * n + 1] = J;
    w.bl[4 * n + 2] = K;
    w.bl[4 * n + 3] = n;
    const std::array<int, 3> ps[6] = {{I, J, K}, {J, I, K}, {I, K, J}, {K, J, I}, {K, I, J}, {J, K, I}};
    for (int s = 0; s < 6; ++s) {
      auto it = idx.find(ps[s]);
      RTCC3_CHECK(it != idx.end(), "triples: window not closed under permutation");
      w.part[6 * n + s] = it->second;
    }
    if (I <= J && J <= K) w.canon.insert(w.canon.end(), {I, J, K, n});
  }
}

}  // namespace

void Triples::build_windows() {
  const int o = d_.o;
  // Two window buffers of nw blocks each (t3 and lambda3, each built and then
  // symmetrised in place) and S; larger windows mean fewer, larger launches.
  // Budget: half the free device memory, at most 48 GiB (of the 288 GB of
  // HBM); when all o^3 blocks fit, one window serves both passes and nothing
  // is built twice.
  size_t free_b = 0, total_b = 0;
  RTCC3_HIP(hipMemGetInfo(&free_b, &total_b));
  const int64_t budget = std::max<int64_t>((int64_t)1 << 30, std::min<int64_t>((int64_t)48 << 30, (int64_t)(free_b / 2)));
  int wmax = (int)std::max<int64_t>(6, budget / (16 * (int64_t)d_.v * d_.v * (2 * pad8(d_.v) + o)));
  if (wcap_ > 0) wmax = std::max(6, std::min(wmax, wcap_));
  // ---- RHS windows: canonical triples i <= j <= k with all their orderings
  std::vector<std::array<int, 3>> cur;
  auto flush = [&]() {
    if (cur.empty()) return;
    Window w;
    finish_window(w, cur);
    rhs_windows_.push_back(w);
    cur.clear();
  };
  for (int i = 0; i < o; ++i)
    for (int j = i; j < o; ++j)
      for (int k = j; k < o; ++k) {
        auto ords = orderings(i, j, k);
        if ((int)(cur.size() + ords.size()) > wmax) flush();
        for (auto& t : ords) cur.push_back(t);
      }
  flush();
  if ((int64_t)o * o * o <= wmax) {
    // ---- every block in one window, in slab order (i fastest, then k, then l):
    // all slabs (., l, k) are contiguous and every block is owned
    std::vector<std::array<int, 3>> all;
    Window w;
    for (int l = 0; l < o; ++l)
      for (int k = 0; k < o; ++k) {
        w.slabs.insert(w.slabs.end(), {0, 0, 0, (int)all.size()});
        for (int i = 0; i < o; ++i) all.push_back({i, l, k});
      }
    finish_window(w, all);
    for (int n = 0; n < w.nw; ++n) w.owned.insert(w.owned.end(), {all[n][0], all[n][1], all[n][2], n});
    den_windows_.push_back(w);
    max_nw_ = 0;
    for (auto& x : rhs_windows_) max_nw_ = std::max(max_nw_, x.nw);
    max_nw_ = std::max(max_nw_, w.nw);
    return;
  }
  // ---- density (pair) windows.  The pairs (l,k), k >= l, of one l are grouped
  // into windows up to the budget; a window holds every ordering of {i,l,k}
  // for all i and its pairs, with the slabs (i,l,k) and (i,k,l) first and in
  // order of i.  A canonical triple (x <= y <= z) is owned by the window of
  // the pair (x,y); each triple is built in at most two windows.
  for (int l = 0; l < o; ++l) {
    int k0 = l;
    while (k0 < o) {
      // grow the pair range [k0, k1) while the union of blocks fits
      int k1 = k0 + 1;
      auto count = [&](int kend) {
        std::map<std::array<int, 3>, int> seen;
        for (int k = k0; k < kend; ++k)
          for (int i = 0; i < o; ++i)
            for (auto& t : orderings(i, l, k)) seen[t] = 1;
        return (int)seen.size();
      };
      while (k1 < o && count(k1 + 1) <= wmax) ++k1;
      std::vector<std::array<int, 3>> bl;
      std::map<std::array<int, 3>, int> seen;
      auto add = [&](std::array<int, 3> t) {
        if (seen.count(t)) return;
        seen[t] = (int)bl.size();
        bl.push_back(t);
      };
      Window w;
      for (int k = k0; k < k1; ++k) {
        w.slabs.insert(w.slabs.end(), {0, 0, 0, (int)bl.size()});
        for (int i = 0; i < o; ++i) {
          RTCC3_CHECK(!seen.count({i, l, k}), "triples: slab block listed twice");
          add({i, l, k});
        }
        if (k != l) {
          w.slabs.insert(w.slabs.end(), {0, 0, 0, (int)bl.size()});
          for (int i = 0; i < o; ++i) {
            RTCC3_CHECK(!seen.count({i, k, l}), "triples: slab block listed twice");
            add({i, k, l});
          }
        }
      }
      for (int k = k0; k < k1; ++k)
        for (int i = 0; i < o; ++i)
          for (auto& t : orderings(i, l, k)) add(t);
      finish_window(w, bl);
      for (int k = k0; k < k1; ++k)
        for (int i = k; i < o; ++i)
          for (auto& t : orderings(i, l, k)) w.owned.insert(w.owned.end(), {t[0], t[1], t[2], seen.at(t)});
      den_windows_.push_back(w);
      k0 = k1;
    }
  }
  max_nw_ = 0;
  for (auto& w : rhs_windows_) max_nw_ = std::max(max_nw_, w.nw);
  for (auto& w : den_windows_) max_nw_ = std::max(max_nw_, w.nw);
}

void Triples::upload(Window& w) {
  auto put = [](int** d, const std::vector<int>& h) {
    RTCC3_HIP(hipMalloc(d, sizeof(int) * h.size()));
    RTCC3_HIP(hipMemcpy(*d, h.data(), sizeof(int) * h.size(), hipMemcpyHostToDevice));
  };
  // group the contraction blocks by J (position 1) and by K (position 2)
  const std::vector<int>& cb = w.owned.empty() ? w.bl : w.owned;
  for (int pos : {1, 2}) {
    Groups& gr = pos == 1 ? w.gJ : w.gK;
    std::map<int, std::vector<int>> by;
    for (size_t e = 0; e < cb.size(); e += 4) by[cb[e + pos]].push_back((int)e);
    gr.key.clear();
    gr.start.assign(1, 0);
    gr.bl.clear();
    gr.max = 0;
    for (auto& kv : by) {
      gr.key.insert(gr.key.end(), {0, 0, 0, 0});
      gr.key[gr.key.size() - 4 + pos] = kv.first;
      for (int e : kv.second) gr.bl.insert(gr.bl.end(), cb.begin() + e, cb.begin() + e + 4);
      gr.start.push_back((int)gr.bl.size() / 4);
      gr.max = std::max(gr.max, (int)kv.second.size());
    }
    put(&gr.d_key, gr.key);
    put(&gr.d_start, gr.start);
    put(&gr.d_bl, gr.bl);
  }
  // The block tables again with the orderings of each occupied triple
  // consecutive: a product that reads an entry's permuted partners then has
  // them read by neighbouring workgroups, which run at the same time and find
  // them in the cache, instead of by workgroups a slab of o^2 blocks away.
  auto orbits = [](const std::vector<int>& t) {
    std::map<std::array<int, 3>, std::vector<int>> by;
    for (size_t e = 0; e < t.size(); e += 4) {
      std::array<int, 3> key{t[e], t[e + 1], t[e + 2]};
      std::sort(key.begin(), key.end());
      by[key].push_back((int)e);
    }
    std::vector<int> out;
    for (auto& kv : by)
      for (int e : kv.second) out.insert(out.end(), t.begin() + e, t.begin() + e + 4);
    return out;
  };
  w.orb = orbits(w.bl);
  put(&w.d_orb, w.orb);
  if (!w.owned.empty()) {
    w.orb_owned = orbits(w.owned);
    put(&w.d_orb_owned, w.orb_owned);
  }
  // The block tables of the build products, sorted so that neighbouring
  // entries share the operand blocks of K and of J (t3) or I (lambda3, S):
  // those 0.8-3 MB blocks then stay in an XCD's L2 cache for the hundreds of
  // entries that read them instead of being fetched again for each entry.
  auto sorted = [](const std::vector<int>& t, int p0, int p1, int p2) {
    std::vector<std::array<int, 4>> x;
    for (size_t e = 0; e < t.size(); e += 4) x.push_back({t[e], t[e + 1], t[e + 2], t[e + 3]});
    std::stable_sort(x.begin(), x.end(), [&](const std::array<int, 4>& a, const std::array<int, 4>& b) {
      return std::make_tuple(a[p0], a[p1], a[p2]) < std::make_tuple(b[p0], b[p1], b[p2]);
    });
    std::vector<int> out;
    for (auto& q : x) out.insert(out.end(), q.begin(), q.end());
    return out;
  };
  w.bk_t3 = sorted(w.bl, 2, 1, 0);
  w.bk_l3 = sorted(w.bl, 2, 0, 1);
  put(&w.d_bk_t3, w.bk_t3);
  put(&w.d_bk_l3, w.bk_l3);
  if (!w.owned.empty()) {
    w.bk_own = sorted(w.owned, 2, 0, 1);
    put(&w.d_bk_own, w.bk_own);
  }
  RTCC3_HIP(hipMalloc(&w.d_bl, sizeof(int) * w.bl.size()));
  RTCC3_HIP(hipMemcpy(w.d_bl, w.bl.data(), sizeof(int) * w.bl.size(), hipMemcpyHostToDevice));
  RTCC3_HIP(hipMalloc(&w.d_part, sizeof(int) * w.part.size()));
  RTCC3_HIP(hipMemcpy(w.d_part, w.part.data(), sizeof(int) * w.part.size(), hipMemcpyHostToDevice));
  if (!w.slabs.empty()) {
    RTCC3_HIP(hipMalloc(&w.d_slabs, sizeof(int) * w.slabs.size()));
    RTCC3_HIP(hipMemcpy(w.d_slabs, w.slabs.data(), sizeof(int) * w.slabs.size(), hipMemcpyHostToDevice));
  }
  RTCC3_HIP(hipMalloc(&w.d_canon, sizeof(int) * w.canon.size()));
  RTCC3_HIP(hipMemcpy(w.d_canon, w.canon.data(), sizeof(int) * w.canon.size(), hipMemcpyHostToDevice));
  if (!w.owned.empty()) {
    RTCC3_HIP(hipMalloc(&w.d_owned, sizeof(int) * w.owned.size()));
    RTCC3_HIP(hipMemcpy(w.d_owned, w.owned.data(), sizeof(int) * w.owned.size(), hipMemcpyHostToDevice));
  }
}

// T1-transformed integral blocks in the layouts the triples contractions read.
void Triples::blocks(Engine& e, const CCSDResult& r) {
  const int64_t o = d_.o, v = d_.v, n = d_.n;
  auto B = [&](char a, char b) {
    return Engine::slice(Engine::slice(r.Bt, 1, a == 'o' ? 0 : o, a == 'o' ? o : n), 2, b == 'o' ? 0 : o,
                         b == 'o' ? o : n);
  };
  auto make = [&](const char* name, std::vector<int64_t> shape) {
    View t = e.tensor(name, shape);
    e.zero(t);
    return t;
  };
  View t;
  t = make("tb_W1", {o, v, v, v});  // (ck|be) at [k][e][b][c]
  e.einsum("Pck,Pbe->kebc", ONE, B('v', 'o'), B('v', 'v'), t);
  t = make("tb_W2", {o, o, v, o});  // -(mk|ai) at [k][i][a][m]
  e.einsum("Pmk,Pai->kiam", R(-1), B('o', 'o'), B('v', 'o'), t);
  t = make("tb_LA", {o, v, v, v});  // -(ib|dc) at [i][d][b][c]
  e.einsum("Pib,Pdc->idbc", R(-1), B('o', 'v'), B('v', 'v'), t);
  t = make("tb_LB", {o, v, v, v});  // 2(db|kc) - (dc|kb) at [k][d][b][c]
  e.einsum("Pdb,Pkc->kdbc", R(2), B('v', 'v'), B('o', 'v'), t);
  e.einsum("Pdc,Pkb->kdbc", R(-1), B('v', 'v'), B('o', 'v'), t);
  t = make("tb_LC", {o, v, o, o});  // (ka|jl) at [k][a][j][l]
  e.einsum("Pka,Pjl->kajl", ONE, B('o', 'v'), B('o', 'o'), t);
  t = make("tb_LD", {o, v, o, o});  // -(2(ia|jl) - (il|ja)) at [i][a][j][l]
  e.einsum("Pia,Pjl->iajl", R(-2), B('o', 'v'), B('o', 'o'), t);
  e.einsum("Pil,Pja->iajl", ONE, B('o', 'o'), B('o', 'v'), t);
  t = make("tb_X2a", {o, v, v, v});  // (ac|ke) at [k][a][c][e]
  e.einsum("Pac,Pke->kace", ONE, B('v', 'v'), B('o', 'v'), t);
  t = make("tb_X2b", {o, o, o, v});  // (ki|mc) at [k][m][i][c]
  e.einsum("Pki,Pmc->kmic", ONE, B('o', 'o'), B('o', 'v'), t);
  t = make("tb_X2c", {o, o, o, v});  // (ki|mc) - 2(mi|kc) at [k][m][i][c] (+ the f~ term below)
  e.einsum("Pki,Pmc->kmic", ONE, B('o', 'o'), B('o', 'v'), t);
  e.einsum("Pmi,Pkc->kmic", R(-2), B('o', 'o'), B('o', 'v'), t);
  if (o <= 15) {
    // The f~ term of X2, sum_c (t[a,b,c] - t[c,b,a]) f~_kc into X2p[I][J], goes through
    // the same gathered product: its second part relabelled (t_IJK[c][b][a] = t_KJI[a][b][c],
    // then I <-> K), both read the block itself, so
    //   X2c[k][m][i][c] += delta_im f~_kc - delta_ik f~_mc.
    auto bcast = [&](int64_t s0, int64_t s1) {  // f~[.][o + c] over (k, m, c) with strides s0, s1
      View x;
      x.nd = 3;
      x.sh[0] = o, x.sh[1] = o, x.sh[2] = v;
      x.st[0] = s0, x.st[1] = s1, x.st[2] = 1;
      x.p = r.F.p + o;
      return x;
    };
    e.axpy(ONE, bcast(n, 0), Engine::diag(t, 1, 2));   // [k][m][m][c] += f~_kc
    e.axpy(R(-1), bcast(0, n), Engine::diag(t, 0, 2));  // [k][m][k][c] -= f~_mc
  }
  t = make("tb_Y2a", {o, v, v, v});  // (da|el) at [l][a][d][e]
  e.einsum("Pda,Pel->lade", ONE, B('v', 'v'), B('v', 'o'), t);
  t = make("tb_Y2b", {o, o, o, v});  // (xi|dk) at [i][k][x][d]
  e.einsum("Pxi,Pdk->ikxd", ONE, B('o', 'o'), B('v', 'o'), t);
  t = make("tb_G1", {o, o, v, v});  // (xc|jd) at [j][x][c][d]
  e.einsum("Pxc,Pjd->jxcd", ONE, B('o', 'v'), B('o', 'v'), t);
  t = make("tb_G5", {o, o, v, v});  // L_jbxc = 2(jb|xc) - (jc|xb) at [j][x][b][c]
  e.einsum("Pjb,Pxc->jxbc", R(2), B('o', 'v'), B('o', 'v'), t);
  e.einsum("Pjc,Pxb->jxbc", R(-1), B('o', 'v'), B('o', 'v'), t);
  t = make("tb_G9", {o, v, v, o});  // (xl|db) at [l][b][d][x]
  e.einsum("Pxl,Pdb->lbdx", ONE, B('o', 'o'), B('v', 'v'), t);
  t = make("tb_G10", {o, v, v, o});  // (dl|xb) at [l][b][d][x]
  e.einsum("Pdl,Pxb->lbdx", ONE, B('v', 'o'), B('o', 'v'), t);
}

void Triples::window_pass(Engine& e, const Window& w, const cplx* y, bool rhs_terms, bool density_terms) {
  const int o = d_.o, v = d_.v;
  const int64_t v2 = (int64_t)v * v, v3 = v2 * v, ov = (int64_t)o * v, oovv = (int64_t)o * o * v2;
  const int64_t ylen = 2 * (ov + oovv);
  const int nw = w.nw;
  hipStream_t s = e.stream;  // t3 side
  hipStream_t s2 = single_ ? s : s2_;  // lambda3 side
  const cplx* t2 = y + ov;
  const cplx* l1 = y + ov + oovv;
  const cplx* l2 = y + 2 * ov + oovv;
  const int64_t t2len = oovv, l2len = oovv;
  (void)ylen;
  // Window blocks are [v][v][vp]: the innermost index is padded to a multiple
  // of 8 so that every row starts on a 128-byte line; the padding stays zero.
  const int vp = pad8(v);
  const int64_t va = (int64_t)v * vp, vb = va * v;  // strides of the first index and of a block
  const int64_t winlen = (int64_t)max_nw_ * vb;
  // The window buffers first: a buffer's first request zero-fills it on the
  // engine stream, which must come before the fork below.
  // The builds write W' into T and L, which the symmetrisation then turns
  // into t3 and lambda3 in place.
  cplx* T = e.tensor("tw_T", {(int64_t)max_nw_, v, v, vp}).p;
  cplx* L = e.tensor("tw_L", {(int64_t)max_nw_, v, v, vp}).p;
  cplx* S = e.tensor("tw_S", {(int64_t)max_nw_, v, v, o}).p;
  RTCC3_HIP(hipEventRecord(ev_fork_, s));
  RTCC3_HIP(hipStreamWaitEvent(s2, ev_fork_, 0));
  auto P = [&](const char* name, std::vector<int64_t> shape) { return e.tensor(name, shape).p; };
  const cplx* gW1 = P("tb_W1", {o, v, v, v});
  const cplx* gW2 = P("tb_W2", {o, o, v, o});
  const cplx* gLA = P("tb_LA", {o, v, v, v});
  const cplx* gLB = P("tb_LB", {o, v, v, v});
  const cplx* gLC = P("tb_LC", {o, v, o, o});
  const cplx* gLD = P("tb_LD", {o, v, o, o});
  const cplx* gX2a = P("tb_X2a", {o, v, v, v});
  const cplx* gX2b = P("tb_X2b", {o, o, o, v});
  const cplx* gX2c = P("tb_X2c", {o, o, o, v});
  const cplx* gY2a = P("tb_Y2a", {o, v, v, v});
  const cplx* gY2b = P("tb_Y2b", {o, o, o, v});
  const cplx* gG1 = P("tb_G1", {o, o, v, v});
  const cplx* gG5 = P("tb_G5", {o, o, v, v});
  const cplx* gG9 = P("tb_G9", {o, v, v, o});
  const cplx* gG10 = P("tb_G10", {o, v, v, o});
  const cplx* Lov = P("Lov", {o, v, o, v});
  const cplx* F = P("F", {(int64_t)d_.n, (int64_t)d_.n});
  const int64_t lOVVV = (int64_t)o * v3, lOOOV = (int64_t)o * o * o * v, lOOVV = oovv;
  const int* bl = w.d_bl;
  const int* blh = w.bl.data();
  const int pr = prec_;

  // Both builds produce W[n][a][(b,c)] in one store-mode product.  A term X
  // whose natural layout is [(a,b)][c] is taken at the cyclically relabelled
  // block instead, Y_ijk^abc = X_jki^bca, which has the layout [a][(b,c)]:
  // P_ijk^abc sums over all simultaneous permutations of (ijk) and (abc), so
  // P Y = P X.
  const int64_t lT2 = t2len, lOVVV_ = lOVVV;
  auto up16 = [](int k) { return (k + 15) / 16 * 16; };
  // Segments start at multiples of 16 (the kernels' K step).
  auto seg = [](GemmDesc::Seg& sg, int k0, int len, const cplx* A, std::initializer_list<int64_t> cA, int64_t sAm,
                int64_t sAk, const cplx* B, std::initializer_list<int64_t> cB, int64_t sBk) {
    sg.k0 = k0;
    sg.len = len;
    sg.A = A;
    std::copy(cA.begin(), cA.end(), sg.cA);
    sg.sAm = sAm;
    sg.sAk = sAk;
    sg.B = B;
    std::copy(cB.begin(), cB.end(), sg.cB);
    sg.sBk = sBk;
    sg.sBn = 1;
  };

  // ---------------- t3 blocks
  {  // W[n][a][(b,c)] = sum_e t2[I][J][a][e] (ck|be)~[K][e][(b,c)]
     //              + sum_m -(mk|ai)~[K][I][a][m] t2[J][m][(b,c)]   (term 2 relabelled)
    GemmDesc g = base(v, (int)v2, up16(v) + o, nw, w.d_bk_t3, pr);
    g.grp = o;  // runs of o entries share K and J
    g.store = 1;
    g.nseg = 2;
    seg(g.seg[0], 0, v, t2, {(int64_t)o * v2, v2, 0, 0}, v, 1, gW1, {0, 0, v3, 0}, v2);
    seg(g.seg[1], up16(v), o, gW2, {(int64_t)v * o, 0, (int64_t)o * v * o, 0}, o, 1, t2, {0, (int64_t)o * v2, 0, 0},
        v2);
    g.C = T;  // C[a][(b,c)] at a*va + b*vp + c
    g.sCm0 = va;
    g.N0 = v;
    g.sCn1 = vp;
    g.sCn0 = 1;
    set4(g.cC, 0, 0, 0, vb);
    const int64_t lA[2] = {lT2, lOOOV}, lB[2] = {lOVVV_, lT2};
    build_event(s);
    prod_seg(e, g, w.bk_t3.data(), lA, lB, winlen, s);
    build_event(s);
    build_flop_ += 8.0 * nw * v * v2 * (v + o);
  }
  RTCC3_HIP(hipEventRecord(ev_t3b_, s));
  launch_sym_cube(T, w.d_canon, (int)w.canon.size() / 4, w.d_part, eps_, o, v, vp, nullptr, nullptr, s);
  if (e.tangent())  // the symmetrisation and the denominator are linear in W'
    launch_sym_cube(e.twin_out(T), w.d_canon, (int)w.canon.size() / 4, w.d_part, eps_, o, v, vp, nullptr, nullptr, s);
  RTCC3_HIP(hipEventRecord(ev_t_, s));  // t3 blocks ready

  // Contractions run over the blocks this window is responsible for: all of
  // them in a plain window, the owned ones in a pair window.
  const bool pairwin = !w.owned.empty() && density_terms;
  const int* cbl = pairwin ? w.d_owned : bl;
  const int* cblh = pairwin ? w.owned.data() : blh;
  const int cn = pairwin ? (int)w.owned.size() / 4 : nw;
  const int* obl = pairwin ? w.d_orb_owned : w.d_orb;  // the same entries, grouped by occupied triple
  const int* oblh = pairwin ? w.orb_owned.data() : w.orb.data();
  if (rhs_terms) {
    // S needs only t2 and integrals: it goes first on the lambda3 side, beside
    // the t3 symmetrisation (memory bound) rather than beside other products
    RTCC3_HIP(hipStreamWaitEvent(s2, ev_t3b_, 0));
    {  // terms 9, 10: S[n][c][(d,x)] = sum_b t2[J][K][c][b] (xI|db)~[I][b][(d,x)]
       //                          + sum_b t2[J][I][c][b] (dK|xb)~[K][b][(d,x)]   (one store-mode product)
      const int* sbl = pairwin ? w.d_bk_own : w.d_bk_l3;  // cbl sorted by (K, I, J)
      const int* sblh = pairwin ? w.bk_own.data() : w.bk_l3.data();
      GemmDesc g = base(v, (int)(o * v), up16(v) + v, cn, sbl, pr);
      g.grp = o;  // runs of o entries share K and I
      g.store = 1;
      g.nseg = 2;
      const int64_t ov2 = (int64_t)o * v2, v2o = v2 * o;
      seg(g.seg[0], 0, v, t2, {0, ov2, v2, 0}, v, 1, gG9, {v2o, 0, 0, 0}, (int64_t)v * o);
      seg(g.seg[1], up16(v), v, t2, {v2, ov2, 0, 0}, v, 1, gG10, {0, 0, v2o, 0}, (int64_t)v * o);
      g.C = S;
      g.sCm0 = (int64_t)v * o;
      g.sCn0 = 1;
      set4(g.cC, 0, 0, 0, v2o);
      const int64_t lS = (int64_t)max_nw_ * v2 * o;
      const int64_t lA[2] = {t2len, t2len}, lB[2] = {lOOVV, lOOVV};
      build_event(s2);  // same kernel as the builds: timed with them
      prod_seg(e, g, sblh, lA, lB, lS, s2);
      build_event(s2);
      build_flop_ += 8.0 * cn * v * (o * v) * (2 * v);
    }
  }

  // ---------------- lambda3 blocks
  {  // W[n][a][(b,c)] = sum_l (ka|jl)~[K][a][J][l] l2[l][I][(b,c)]
     //              - sum_l Lt_ijal[I][a][J][l] l2[l][K][(b,c)]
     //              + sum_d l2[J][K][a][d] -(ib|dc)~[I][d][(b,c)]                (relabelled)
     //              + sum_d l2[I][J][a][d] (2(db|kc) - (dc|kb))~[K][d][(b,c)]    (relabelled)
    const int k1 = up16(o), k2 = 2 * up16(o), k3 = 2 * up16(o) + up16(v);
    GemmDesc g = base(v, (int)v2, k3 + v, nw, w.d_bk_l3, pr);
    g.grp = o;  // runs of o entries share K and I
    g.store = 1;
    g.nseg = 4;
    const int64_t oo = (int64_t)o * o, ov2 = (int64_t)o * v2;
    seg(g.seg[0], 0, o, gLC, {0, o, (int64_t)v * oo, 0}, oo, 1, l2, {v2, 0, 0, 0}, ov2);
    seg(g.seg[1], k1, o, gLD, {(int64_t)v * oo, o, 0, 0}, oo, 1, l2, {0, 0, v2, 0}, ov2);
    seg(g.seg[2], k2, v, l2, {0, ov2, v2, 0}, v, 1, gLA, {v3, 0, 0, 0}, v2);
    seg(g.seg[3], k3, v, l2, {ov2, v2, 0, 0}, v, 1, gLB, {0, 0, v3, 0}, v2);
    g.C = L;
    g.sCm0 = va;
    g.N0 = v;
    g.sCn1 = vp;
    g.sCn0 = 1;
    set4(g.cC, 0, 0, 0, vb);
    const int64_t lLC = (int64_t)o * v * o * o;
    const int64_t lA[4] = {lLC, lLC, l2len, l2len}, lB[4] = {l2len, l2len, lOVVV_, lOVVV_};
    RTCC3_HIP(hipStreamWaitEvent(s2, ev_t3b_, 0));  // after the t3 build (a no-op when S went first)
    build_event(s2);
    prod_seg(e, g, w.bk_l3.data(), lA, lB, winlen, s2);
    build_event(s2);
    build_flop_ += 8.0 * nw * v * v2 * (2 * o + 2 * v);
    RTCC3_HIP(hipEventRecord(ev_l3b_, s2));
    if (beside_) {
      side_done_ = (*beside_)(ev_l3b_);
      beside_ = nullptr;
    }
  }
  {  // P_ijk^abc and the denominator; the terms without a summation index are added per source
    LamElem le{Lov, F, l1, l2};
    launch_sym_cube(L, w.d_canon, (int)w.canon.size() / 4, w.d_part, eps_, o, v, vp, &le, nullptr, s2);
    if (e.tangent()) {
      // the bracket terms' derivative: L l1' + f~' l2 + f~ l2' (L is invariant
      // under the T1 transformation: its twin is zero)
      RTCC3_CHECK(!e.twin(Lov), "triples: L_iajb has a derivative");
      LamElem d0{Lov, e.twin(F), e.twin(l1), l2}, d1{nullptr, F, nullptr, e.twin(l2)};
      launch_sym_cube(e.twin_out(L), w.d_canon, (int)w.canon.size() / 4, w.d_part, eps_, o, v, vp, &d0,
                      d1.l2 ? &d1 : nullptr, s2);
    }
  }
  RTCC3_HIP(hipEventRecord(ev_l_, s2));  // lambda3 blocks ready
  launches_ += 4;

  if (rhs_terms) {
    cplx* X1 = P("tr_X1", {o, v});
    cplx* X2p = P("tr_X2p", {o, o, v, v});
    cplx* Y1 = P("tr_Y1", {o, v});
    cplx* Y2p = P("tr_Y2p", {o, o, v, v});
    cplx* Z34 = P("tr_Z34", {o, v});
    cplx* R15 = P("tr_R15", {o, o, v, o});
    cplx* R2t = P("tr_R2", {o, o, v, o});
    cplx* R6 = P("tr_R6", {o, o, v, o});
    cplx* R8 = P("tr_R8", {o, o, v, o});
    cplx* Zi = P("tr_Zi", {o, v, v, v});
    cplx* R12 = P("tr_R12", {o, o, o, v});
    const int64_t lR = (int64_t)o * o * v * o;

    // X1, the f~ term of X2 and Z34 (terms 3 and 4 of Y1): with o <= 15 they ride
    // along with products that read the block anyway (tail columns of the Y1
    // product below; the f~ term inside tb_X2c); else one sweep per block
    const bool tails = o <= 15;
    if (!tails) {
      RTCC3_CHECK(!e.tangent(), "triples: derivatives need o <= 15");
      launch_small_t3(T, cbl, cn, Lov, F, l2, X1, X2p, Z34, o, v, vp, 3, s);
    }
    // the t3 side's products are bound by the matrix cores like the lambda3
    // build: they start once it is done
    RTCC3_HIP(hipStreamWaitEvent(s, ev_l3b_, 0));
    // The combinations of X2 in terms of the window's blocks: with
    // t_{sigma(ijk)}^{sigma(abc)} = t_ijk^abc, for the block (I,J,K)
    //   Z1[b][c][e] = 2t[c,b,e] - t[c,e,b] - t[e,b,c] = (2 T_JIK - T_KIJ - T_JKI)[b][c][e]
    //   Zh[a][b][c] = 2t[c,b,a] - t[b,c,a] - t[a,b,c] = (2 T_KJI - T_KIJ - T_IJK)[a][b][c]
    // (window orderings: 0 IJK, 1 JIK, 2 IKJ, 3 KJI, 4 KIJ, 5 JKI).
    auto combine = [&](GemmDesc& g, int on, int p0, int p1, int p2) {
      g.comb_n = 3;
      g.comb_on = on;
      g.part = w.d_part;
      g.comb_perm[0] = p0;
      g.comb_perm[1] = p1;
      g.comb_perm[2] = p2;
      g.comb_w[0] = 2.0;
      g.comb_w[1] = -1.0;
      g.comb_w[2] = -1.0;
      g.comb_stride = vb;
    };
    {  // X2: sum_ce Z1[b][(c,e)] (ac|ke)~ into X2p[I][J][a][b], with (c,e) contiguous:
       //   Z1[b][c][e] = (2 T_JIK - T_KIJ - T_JKI)[b][c][e]
      GemmDesc g = base(v, v, (int)v2, cn, obl, pr);
      g.atomic = 1;
      g.K0 = v;  // k = (c,e)
      g.A = gX2a;
      g.sAm0 = v2;
      g.sAk1 = v;
      g.sAk0 = 1;
      set4(g.cA, 0, 0, v3, 0);
      g.B = T;  // B[(c,e)][b] = Z1[b][(c,e)]
      g.sBk1 = vp;
      g.sBk0 = 1;
      g.sBn0 = va;
      set4(g.cB, 0, 0, 0, vb);
      combine(g, 1, 1, 4, 5);
      g.C = X2p;
      g.sCm0 = v;
      g.sCn0 = 1;
      set4(g.cC, (int64_t)o * v2, v2, 0, 0);
      prod(e, g, oblh, lOVVV, winlen, oovv, s);
    }
    // X2 -= sum_c Zh[(a,b)][c] G[K][I][c][x] into X2p[x][J], G[k][m][c][x] = (kx|mc)~.
    // The contraction set holds every ordering of its triples, so each term of
    // Zh can be summed with its occupied labels renamed until it reads the
    // block itself:
    //   -2 T_KJI G[K][I] -> -2 T_IJK G[I][K]   (I <-> K)
    //      T_KIJ G[K][I] ->    T_IJK G[I][J] into X2p[x][K]   ((K,I,J) -> (I,J,K))
    //      T_IJK G[K][I] stays.
    // Two gathered products, over the blocks of each J and of each K, without atomics:
    auto x2b = [&](const cplx* Bp, const int64_t* cb, const int64_t* cc, const Groups& gr) {
      GemmDesc g = base((int)v2, o, v * gr.max, 0, nullptr, pr);
      g.K0 = v;
      g.M0 = v;  // m = (a,b)
      g.A = T;   // A[(a,b)][c] = T_IJK[a][b][c]
      g.sAm1 = va;
      g.sAm0 = vp;
      g.sAk0 = 1;
      set4(g.cA, 0, 0, 0, vb);
      g.B = Bp;
      g.sBk0 = 1;
      g.sBn0 = v;
      std::memcpy(g.cB, cb, sizeof(g.cB));
      g.C = X2p;
      g.sCm1 = v;
      g.sCm0 = 1;
      g.sCn0 = (int64_t)o * v2;
      std::memcpy(g.cC, cc, sizeof(g.cC));
      prod_gather(e, g, gr, winlen, lOOOV, oovv, s);
    };
    {
      // (G[K][I] - 2 G[I][K]) is tb_X2c at [K][I]; G[I][J] is tb_X2b at [I][J]
      const int64_t cbJ[4] = {(int64_t)o * v, 0, (int64_t)o * o * v, 0}, ccJ[4] = {0, v2, 0, 0};
      const int64_t cbK[4] = {(int64_t)o * o * v, (int64_t)o * v, 0, 0}, ccK[4] = {0, 0, v2, 0};
      x2b(gX2c, cbJ, ccJ, w.gJ);
      x2b(gX2b, cbK, ccK, w.gK);
    }
    {  // Y2: sum_de (da|eK)~ lambda[d][b][e] into Y2p[I][J][a][b]; lambda_IJK[d][b][e] =
       // lambda_JIK[b][d][e], read with (d,e) contiguous
      GemmDesc g = base(v, v, (int)v2, cn, cbl, pr);
      g.atomic = 1;
      g.K0 = v;  // k = (d,e)
      g.A = gY2a;
      g.sAm0 = v2;
      g.sAk1 = v;
      g.sAk0 = 1;
      set4(g.cA, 0, 0, v3, 0);
      g.B = L;
      g.sBk1 = vp;
      g.sBk0 = 1;
      g.sBn0 = va;
      set4(g.cB, 0, 0, 0, vb);
      g.comb_n = 1;
      g.comb_on = 1;
      g.part = w.d_part;
      g.comb_perm[0] = 1;
      g.comb_stride = vb;
      g.C = Y2p;
      g.sCm0 = v;
      g.sCn0 = 1;
      set4(g.cC, (int64_t)o * v2, v2, 0, 0);
      prod(e, g, cblh, lOVVV, winlen, oovv, s2);
    }
    {  // Y2: -sum_d lambda[(a,b)][d] (xI|dK)~ into Y2p[x][J], summed over the blocks of each J
      GemmDesc g = base((int)v2, o, v * w.gJ.max, 0, nullptr, pr);
      g.K0 = v;
      g.M0 = v;  // m = (a,b)
      g.alpha = R(-1);
      g.A = L;
      g.sAm1 = va;
      g.sAm0 = vp;
      g.sAk0 = 1;
      set4(g.cA, 0, 0, 0, vb);
      g.B = gY2b;
      g.sBk0 = 1;
      g.sBn0 = v;
      set4(g.cB, (int64_t)o * o * v, 0, (int64_t)o * v, 0);
      g.C = Y2p;
      g.sCm1 = v;
      g.sCm0 = 1;
      g.sCn0 = (int64_t)o * v2;
      set4(g.cC, 0, v2, 0, 0);
      prod_gather(e, g, w.gJ, winlen, lOOOV, oovv, s2);
    }
    // Products that read one block of the window as A[m][(k,l)] (M = v,
    // K = v^2, unit stride along (k,l)) and differ in B and C run as column
    // segments of one product: the block is read once for all of them.  A
    // product wider than 16 columns (o > 16) takes several segments, and more
    // than four segments take several launches.
    struct SegSpec {
      GemmDesc::ColSeg c;
      int64_t lenB, lenC, tlenB, tlenC;  // lengths of the B and C tensors (and the tail's)
    };
    auto seg_product = [&](const cplx* X, const std::vector<SegSpec>& specs, hipStream_t st) {
      std::vector<SegSpec> parts;
      for (const SegSpec& sp : specs)
        for (int c0 = 0; c0 < sp.c.n; c0 += 16) {
          SegSpec q = sp;
          q.c.n = std::min(16, sp.c.n - c0);
          q.c.B = sp.c.B + c0 * sp.c.sBn;
          q.lenB = sp.lenB - c0 * sp.c.sBn;
          q.c.C = sp.c.C + c0 * sp.c.sCn;
          q.lenC = sp.lenC - c0 * sp.c.sCn;
          if (c0 > 0) q.c.tB = nullptr, q.c.tC = nullptr;
          parts.push_back(q);
        }
      for (size_t p0 = 0; p0 < parts.size(); p0 += 4) {
        const int ns = (int)std::min<size_t>(4, parts.size() - p0);
        GemmDesc g = base(v, 16 * ns, (int)v2, cn, cbl, pr);
        g.atomic = 1;
        g.A = X;  // A[a][(b,c)] at a*va + b*vp + c; the segments' B read k = (b,c) flattened
        g.K0 = v;
        g.sAm0 = va;
        g.sAk1 = vp;
        g.sAk0 = 1;
        set4(g.cA, 0, 0, 0, vb);
        g.ncs = ns;
        int64_t lenB[8] = {0}, lenC[8] = {0};
        for (int t = 0; t < ns; ++t) {
          const SegSpec& q = parts[p0 + t];
          g.cs[t] = q.c;
          lenB[t] = q.lenB;
          lenC[t] = q.lenC;
          lenB[4 + t] = q.tlenB;
          lenC[4 + t] = q.tlenC;
        }
        prod_colseg(e, g, cblh, winlen, lenB, lenC, st);
      }
    };
    auto cseg = [&](const cplx* Bp, std::initializer_list<int64_t> cb, int64_t sbk, int64_t sbn, cplx* Cp,
                    std::initializer_list<int64_t> cc, int64_t scm, int64_t scn, double alpha) {
      GemmDesc::ColSeg c;
      std::memset(&c, 0, sizeof(c));
      c.n = o;
      c.B = Bp;
      std::copy(cb.begin(), cb.end(), c.cB);
      c.sBk = sbk;
      c.sBn = sbn;
      c.C = Cp;
      std::copy(cc.begin(), cc.end(), c.cC);
      c.sCm = scm;
      c.sCn = scn;
      c.alpha = R(alpha);
      return c;
    };
    auto tail = [&](GemmDesc::ColSeg& c, const cplx* Bp, std::initializer_list<int64_t> cb, cplx* Cp,
                    std::initializer_list<int64_t> cc, double alpha) {
      c.tB = Bp;
      std::copy(cb.begin(), cb.end(), c.tcB);
      c.tsBk = 1;
      c.tC = Cp;
      std::copy(cc.begin(), cc.end(), c.tcC);
      c.tsCm = 1;
      c.talpha = R(alpha);
    };
    {  // Y1 terms 1, 2, 5, 6: per block (j,k,l) = (I,J,K), intermediates C[b][x] = sum_(c,d) t[b][(c,d)] B[(c,d)][x].
       // Term 5 sums t[(b,c)][d] = t_KIJ[d][(b,c)] over the blocks; with the labels renamed
       // ((K,I,J) -> (I,J,K)) it reads the block itself, into R15[K][I] with G5[J].
      const int64_t ovo = (int64_t)o * v * o, vo = (int64_t)v * o, ov2 = (int64_t)o * v2;
      GemmDesc::ColSeg c1 = cseg(gG1, {ov2, 0, 0, 0}, 1, v2, R15, {0, ovo, vo, 0}, o, 1, 1.0);   // term 1: (xc|Id)
      GemmDesc::ColSeg c5 = cseg(gG5, {0, ov2, 0, 0}, 1, v2, R15, {vo, 0, ovo, 0}, o, 1, -1.0);  // term 5: L_Ibxc
      GemmDesc::ColSeg c2 = cseg(l2, {v2, 0, 0, 0}, 1, ov2, R2t, {0, ovo, vo, 0}, o, 1, 1.0);    // term 2: l2[x][I]
      GemmDesc::ColSeg c6 = cseg(l2, {0, 0, v2, 0}, 1, ov2, R6, {ovo, vo, 0, 0}, o, 1, 1.0);     // term 6: l2[x][K]
      if (tails) {
        // X1[I][a] += sum_bc t[a][b][c] L_JbKc, and -sum_bc t[c][b][a] L_JbKc relabelled
        // (t_IJK[c][b][a] = t_KJI[a][b][c], then I <-> K) into X1[K] with L_JbIc;
        // Z34[I][a] += sum_bc t[a][b][c] l2[J][K][b][c], and -sum_bc t[b][a][c] l2[J][K][b][c]
        // relabelled (t_IJK[b][a][c] = t_JIK[a][b][c], then I <-> J) into Z34[J] with l2[I][K].
        // L_JbKc = (tb_G5)[J][K][b][c].
        tail(c1, gG5, {0, ov2, v2, 0}, X1, {v, 0, 0, 0}, 1.0);
        tail(c5, gG5, {v2, ov2, 0, 0}, X1, {0, 0, v, 0}, -1.0);
        tail(c2, l2, {0, ov2, v2, 0}, Z34, {v, 0, 0, 0}, 1.0);
        tail(c6, l2, {ov2, 0, v2, 0}, Z34, {0, v, 0, 0}, -1.0);
      }
      seg_product(T,
                  {{c1, lOOVV, lR, lOOVV, ov}, {c5, lOOVV, lR, lOOVV, ov}, {c2, l2len, lR, l2len, ov},
                   {c6, l2len, lR, l2len, ov}},
                  s);
    }
    {  // One column-segment product over lambda_n[a][(b,c)] (S is ready: same stream, earlier):
       //  terms 7, 8: Q[d][j] = sum_bc lambda[(b,c)][d] t2[j][J][(b,c)] into R8[I][K]; with
       //    lambda[b][c][d] = lambda_KIJ[d][b][c] and the labels renamed ((K,I,J) -> (I,J,K)):
       //    sum_bc lambda_n[d][(b,c)] t2[j][K][(b,c)] into R8[J][I]
       //    (the term-7 intermediate R7[K][I] is the same sum with the first two indices swapped);
       //  Y1[x][a] -= sum_(c,d) lambda_n[a][(c,d)] S[n][(c,d)][x];
       //  term 12: R12[I][j][J][a] += sum_bc lambda_n[a][(b,c)] t2[j][K][(b,c)]   (block (l,m,k) = (I,J,K)).
      const int64_t ovo = (int64_t)o * v * o, vo = (int64_t)v * o, ov2 = (int64_t)o * v2;
      const int64_t lS = (int64_t)max_nw_ * v2 * o;
      const int64_t lR12 = (int64_t)o * o * o * v;
      seg_product(L,
                  {{cseg(t2, {0, 0, v2, 0}, 1, ov2, R8, {vo, ovo, 0, 0}, o, 1, 1.0), t2len, lR, 0, 0},
                   {cseg(S, {0, 0, 0, v2 * o}, o, 1, Y1, {0, 0, 0, 0}, 1, v, -1.0), lS, ov, 0, 0},
                   {cseg(t2, {0, 0, v2, 0}, 1, ov2, R12, {(int64_t)o * o * v, v, 0, 0}, 1, vo, 1.0), t2len, lR12, 0, 0}},
                  s2);
    }
    {  // term 11: Zi[J][b][(d,e)] += sum_c t2[K][I][b][c] lambda[c][(d,e)]   (block (k,i,j) = (I,J,K)),
       // summed over the blocks of each J
      GemmDesc g = base(v, (int)v2, v * w.gJ.max, 0, nullptr, pr);
      g.K0 = v;
      g.A = t2;
      g.sAm0 = v;
      g.sAk0 = 1;
      set4(g.cA, v2, 0, (int64_t)o * v2, 0);
      g.N0 = v;  // n = (d,e)
      g.B = L;
      g.sBk0 = va;
      g.sBn1 = vp;
      g.sBn0 = 1;
      set4(g.cB, 0, 0, 0, vb);
      g.C = Zi;
      g.sCm0 = v2;
      g.sCn1 = v;
      g.sCn0 = 1;
      set4(g.cC, 0, v3, 0, 0);
      prod_gather(e, g, w.gJ, t2len, winlen, lOVVV, s2);
    }
    launches_ += tails ? 9 : 10;
  }

  // the density terms read t3 and lambda3: join the lambda3 side's blocks
  if (density_terms) RTCC3_HIP(hipStreamWaitEvent(s, ev_l_, 0));
  if (density_terms && !w.owned.empty()) {
    const int no = (int)w.owned.size() / 4;
    cplx* Dab = P("td_Dab", {v, v});
    cplx* Z34 = P("td_Z34", {o, v});
    cplx* Rd = P("td_Rd", {o, o, v, o});
    {  // D_ab += 1/2 sum_{(d,c)} lambda[a][(d,c)] t[b][(d,c)]
      GemmDesc g = base(v, v, (int)v2, no, w.d_owned, pr);
      g.atomic = 1;
      g.alpha = R(0.5);
      g.K0 = v;  // k = (d,c)
      g.A = L;
      g.sAm0 = va;
      g.sAk1 = vp;
      g.sAk0 = 1;
      set4(g.cA, 0, 0, 0, vb);
      g.B = T;
      g.sBk1 = vp;
      g.sBk0 = 1;
      g.sBn0 = va;
      set4(g.cB, 0, 0, 0, vb);
      g.C = Dab;
      g.sCm0 = v;
      g.sCn0 = 1;
      prod(e, g, w.owned.data(), winlen, winlen, v2, s);
    }
    // D_ia first term: sum_bc (t[a,b,c] - t[b,a,c]) l2[J,K,b,c]; it equals the
    // Y1 intermediate Z34 when the same pass also evaluates the right-hand side
    if (!rhs_terms) {
      RTCC3_CHECK(!e.tangent(), "triples: derivatives of the density need the right-hand side pass");
      launch_small_t3(T, w.d_owned, no, Lov, F, l2, nullptr, nullptr, Z34, o, v, vp, 2, s);
    }
    {  // D_ia second term: Rd[J][I][b][x] += sum_cd lambda[b][(c,d)] t2[x][K][(c,d)]
      GemmDesc g = base(v, o, (int)v2, no, w.d_owned, pr);
      g.atomic = 1;
      g.K0 = v;  // k = (c,d)
      g.A = L;
      g.sAm0 = va;
      g.sAk1 = vp;
      g.sAk0 = 1;
      set4(g.cA, 0, 0, 0, vb);
      g.B = t2;
      g.sBk1 = v;
      g.sBk0 = 1;
      g.sBn0 = (int64_t)o * v2;
      set4(g.cB, 0, 0, v2, 0);
      g.C = Rd;
      g.sCm0 = o;
      g.sCn0 = 1;
      set4(g.cC, (int64_t)v * o, (int64_t)o * v * o, 0, 0);
      prod(e, g, w.owned.data(), winlen, t2len, (int64_t)o * o * v * o, s);
    }
  }
  if (density_terms && !w.slabs.empty()) {
    // D_ij += -1/2 sum_abc t_{ilk} lambda_{jlk}, one batch entry per slab (., l, k);
    // on the lambda3 side, once the t3 blocks are ready
    RTCC3_HIP(hipStreamWaitEvent(s2, ev_t_, 0));
    cplx* Dij = P("td_Dij", {o, o});
    const int nslab = (int)w.slabs.size() / 4;
    if (o <= 16) {
      for (int q = 0; q < nslab; ++q)
        RTCC3_CHECK(w.slabs[4 * q + 3] >= 0 && (int64_t)(w.slabs[4 * q + 3] + o) * vb <= winlen,
                    "triples: slab out of bounds");
      // whole padded blocks: the padding is zero and adds nothing
      launch_gram(T, L, w.d_slabs, nslab, o, vb, R(-0.5), Dij, s2);
      if (e.tangent()) {
        const cplx *Tt = e.twin(T), *Lt = e.twin(L);
        if (Tt || Lt) {
          cplx* Dt = e.twin_out(Dij);
          if (Tt) launch_gram(Tt, L, w.d_slabs, nslab, o, vb, R(-0.5), Dt, s2);
          if (Lt) launch_gram(T, Lt, w.d_slabs, nslab, o, vb, R(-0.5), Dt, s2);
        }
      }
    } else {
      GemmDesc g = base(o, o, (int)vb, nslab, w.d_slabs, pr);  // whole padded blocks (zero padding)
      g.atomic = 1;
      g.alpha = R(-0.5);
      g.A = T;
      g.sAm0 = vb;
      g.sAk0 = 1;
      set4(g.cA, 0, 0, 0, vb);
      g.B = L;
      g.sBk0 = 1;
      g.sBn0 = vb;
      set4(g.cB, 0, 0, 0, vb);
      g.C = Dij;
      g.sCm0 = o;
      g.sCn0 = 1;
      prod(e, g, w.slabs.data(), winlen, winlen, (int64_t)o * o, s2);
    }
  }
  // the next window reuses every window buffer: join the lambda3 side
  RTCC3_HIP(hipEventRecord(ev_join_, s2));
  RTCC3_HIP(hipStreamWaitEvent(s, ev_join_, 0));
}

void Triples::build_event(hipStream_t s) {
  if (!timing_on_) return;
  // pairs: a full pool is folded before a pair starts
  if (nbev_ % 2 == 0 && nbev_ + 2 > (int)bev_.size()) fold_timing();
  RTCC3_HIP(hipEventRecord(bev_[nbev_++], s));
}

TriplesOut Triples::run(Engine& e, const Dims& d, const CCSDResult& r, const cplx* y, bool want_density,
                        const Beside& beside, hipEvent_t ready) {
  const int64_t o = d.o, v = d.v;
  const int64_t ov = o * v, oovv = o * o * v * v;
  hipStream_t s = e.stream;
  if (timing_on_) {
    if (nrev_ + 2 > (int)rev_.size()) fold_timing();
    RTCC3_HIP(hipEventRecord(rev_[nrev_++], s));
  }
  blocks(e, r);
  beside_ = beside ? &beside : nullptr;
  side_done_ = nullptr;
  // accumulators
  const char* names[] = {"tr_X1", "tr_X2p", "tr_Y1", "tr_Y2p", "tr_Z34", "tr_R15",
                         "tr_R2", "tr_R6", "tr_R8", "tr_Zi",  "tr_R12"};
  std::vector<std::vector<int64_t>> shapes = {{o, v},       {o, o, v, v}, {o, v},       {o, o, v, v},
                                              {o, v},       {o, o, v, o}, {o, o, v, o}, {o, o, v, o},
                                              {o, o, v, o}, {o, v, v, v}, {o, o, o, v}};
  for (size_t i = 0; i < shapes.size(); ++i) e.zero(e.tensor(names[i], shapes[i]));
  if (want_density) {
    View Dij = e.tensor("td_Dij", {o, o}), Dab = e.tensor("td_Dab", {v, v}), Rd = e.tensor("td_Rd", {o, o, v, o});
    e.zero(Dij);
    e.zero(Dab);
    e.zero(Rd);
    // one pass over the pair windows: right-hand side for the owned blocks, density terms
    for (auto& w : den_windows_) window_pass(e, w, y, true, true);
  } else {
    for (auto& w : rhs_windows_) window_pass(e, w, y, true, false);
  }

  if (beside_) {  // no window ran (nothing to overlap): start the side work here
    RTCC3_HIP(hipEventRecord(ev_l3b_, s));
    side_done_ = (*beside_)(ev_l3b_);
    beside_ = nullptr;
  }
  // the final contractions read blocks of the CCSD residual (and use this
  // stream's own scratch): they need not wait for the work beside
  if (ready) RTCC3_HIP(hipStreamWaitEvent(s, ready, 0));
  // ---- final contractions of the Y1 intermediates
  View Y1 = e.tensor("tr_Y1", {o, v});
  View l2 = Engine::raw(const_cast<cplx*>(y) + 2 * ov + oovv, {o, o, v, v});
  View Lov = e.tensor("Lov", {o, v, o, v});
  View g_ovov = e.tensor("g_ovov", {o, v, o, v});
  View g_oovv = e.tensor("g_oovv", {o, o, v, v});
  View g_voov = e.tensor("g_voov", {v, o, o, v});
  View g_vvvv = e.tensor("g_vvvv", {v, v, v, v});
  View g_oooo = e.tensor("g_oooo", {o, o, o, o});
  e.einsum("klbx,klab->xa", ONE, e.tensor("tr_R15", {o, o, v, o}), l2, Y1);
  e.einsum("klbx,kalb->xa", ONE, e.tensor("tr_R2", {o, o, v, o}), g_ovov, Y1);
  e.einsum("jkbx,kajb->xa", R(-1), e.tensor("tr_R6", {o, o, v, o}), Lov, Y1);
  e.einsum("xajb,jb->xa", ONE, Lov, e.tensor("tr_Z34", {o, v}), Y1);
  e.einsum("lidj,jlda->ia", R(-1), e.tensor("tr_R8", {o, o, v, o}), g_oovv, Y1);
  e.einsum("ildj,dlja->ia", R(-1), e.tensor("tr_R8", {o, o, v, o}), g_voov, Y1);
  e.einsum("ibde,daeb->ia", ONE, e.tensor("tr_Zi", {o, v, v, v}), g_vvvv, Y1);
  e.einsum("xljm,ljma->xa", ONE, g_oooo, e.tensor("tr_R12", {o, o, o, v}), Y1);

  TriplesOut out;
  out.X1 = e.tensor("tr_X1", {o, v});
  out.Y1 = Y1;
  // P_ij^ab symmetrisation of X2 and Y2
  View X2 = e.tensor("tr_X2", {o, o, v, v});
  e.zero(X2);
  View X2p = e.tensor("tr_X2p", {o, o, v, v});
  e.axpy(ONE, X2p, X2);
  e.axpy(ONE, Engine::permute(X2p, {1, 0, 3, 2}), X2);
  View Y2 = e.tensor("tr_Y2", {o, o, v, v});
  e.zero(Y2);
  View Y2p = e.tensor("tr_Y2p", {o, o, v, v});
  e.axpy(ONE, Y2p, Y2);
  e.axpy(ONE, Engine::permute(Y2p, {1, 0, 3, 2}), Y2);
  out.X2 = X2;
  out.Y2 = Y2;

  if (want_density) {
    View Dij = e.tensor("td_Dij", {o, o}), Dab = e.tensor("td_Dab", {v, v}), Rd = e.tensor("td_Rd", {o, o, v, o});
    View Z34 = e.tensor("tr_Z34", {o, v});
    View Dia = e.tensor("td_Dia", {o, v});
    e.zero(Dia);
    e.axpy(ONE, Z34, Dia);
    View t2 = Engine::raw(const_cast<cplx*>(y) + ov, {o, o, v, v});
    e.einsum("kjbx,kjab->xa", R(-1), Rd, t2, Dia);
    out.Dij = Dij;
    out.Dab = Dab;
    out.Dia = Dia;
  }
  if (timing_on_) RTCC3_HIP(hipEventRecord(rev_[nrev_++], s));
  return out;
}

}  // namespace rtcc3
