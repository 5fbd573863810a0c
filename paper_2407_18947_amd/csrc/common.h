// Shared host/device definitions of the RT-CC3 library.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <stdexcept>
#include <string>

namespace rtcc3 {

struct cplx {
  double re, im;
};

// Host-side error carrying an RTCC3_* code.
struct Error : std::runtime_error {
  int code;
  Error(int c, const std::string& m) : std::runtime_error(m), code(c) {}
};

// Message of the last failed context-free call of this thread (rtcc3_last_error(NULL)).
void set_thread_error(const std::string& msg);

#define RTCC3_HIP(call)                                                                       \
  do {                                                                                        \
    hipError_t e_ = (call);                                                                   \
    if (e_ != hipSuccess)                                                                     \
      throw ::rtcc3::Error(-3, std::string(#call) + ": " + hipGetErrorString(e_));            \
  } while (0)

#define RTCC3_CHECK(cond, msg)                                                                \
  do {                                                                                        \
    if (!(cond)) throw ::rtcc3::Error(-1, msg);                                               \
  } while (0)

// ---------------------------------------------------------------------------
// Kernel entry points (kernels.hip)
// ---------------------------------------------------------------------------

// Batched complex GEMM: C[b][m][n] += alpha * sum_k A[b][m][k] B[b][k][n].
// Each of M, N, K is split in two levels (m = m1*M0 + m0, ...) with its own
// element strides, so a tensor index group made of two runs of contiguous
// indices needs no copy.  Batch entry b starts at A + b*sAb (same for B, C),
// or, when a block table bl is given (4 ints per entry: I, J, K, n), at
//   A + cA[0]*I + cA[1]*J + cA[2]*K + cA[3]*n   (same for B and C).
// atomic: accumulate with atomics (several batch entries may share C).
// prec: RTCC3_PREC_FP64: FP64 MFMA; RTCC3_PREC_FP32: operands rounded to FP32,
// FP32 MFMA and accumulate; RTCC3_PREC_BF16X3 / BF16X2: operands split into
// three / two bf16 slices, bf16 MFMA with FP32 accumulate.
enum { RTCC3_PREC_FP64 = 0, RTCC3_PREC_FP32 = 1, RTCC3_PREC_BF16X3 = 2, RTCC3_PREC_BF16X2 = 3 };
struct GemmDesc {
  int M, N, K, batch;
  int M0, N0, K0;
  const cplx* A;
  int64_t sAm1, sAm0, sAk1, sAk0, sAb;
  const cplx* B;
  int64_t sBk1, sBk0, sBn1, sBn0, sBb;
  cplx* C;
  int64_t sCm1, sCm0, sCn1, sCn0, sCb;
  const int* bl;
  int64_t cA[4], cB[4], cC[4];
  cplx alpha;
  int atomic;
  int prec;
  // K segments (nseg > 0, block table required): the contraction runs over
  // consecutive segments, segment s covering k in [seg[s].k0, seg[s].k0 + len)
  // with its own operands
  //   A_s[m][r] = seg[s].A[cA.(I,J,K,n) + m*sAm + r*sAk],
  //   B_s[r][n] = seg[s].B[cB.(I,J,K,n) + r*sBk + n*sBn],   r = k - seg[s].k0,
  // so one product sums terms whose operands live in different tensors.
  // The plain A/B fields and the M0/K0 splits are then unused (M0 = M); N0
  // (with sCn1) splits the columns of C only, B reads the flattened n.
  struct Seg {
    int k0;   // first k; a multiple of 16, so that a K step of 16 lies in one segment
    int len;  // contraction length (k0 + len <= next k0; the gap reads as zero)
    const cplx* A;
    int64_t cA[4], sAm, sAk;
    const cplx* B;
    int64_t cB[4], sBk, sBn;
  };
  int nseg;
  Seg seg[4];
  // store = 1: C = alpha*AB without reading C (no split-K, not atomic).
  int store;
  // A bf16-split precision runs unsegmented products in FP32 unless
  // force_prec is set (self-tests of the split kernel).
  int force_prec;
  // grp > 1 (segmented store products): workgroups walk groups of grp
  // consecutive batch entries column tile by column tile, so the entries of a
  // group (which share their large operand blocks) read each 64-column slice
  // of those blocks one after another, from one XCD's L2.
  int grp;
  // Combined operand (comb_n = 3, block table required, A read k-fast and B
  // k-fast): operand A (comb_on = 0) or B (comb_on = 1) of batch entry b is
  //   sum_s comb_w[s] * X[part[6*n + comb_perm[s]]*comb_stride + offset],  n = bl[4*b + 3],
  // in place of its block-table offset; e.g. a linear combination of a block
  // and blocks of permuted occupied triples read at the same element offset.
  // comb_n = 1 (B only): B is the single block part[6*n + comb_perm[0]].
  int comb_n, comb_on;
  const int* part;
  int comb_perm[3];
  double comb_w[3];
  int64_t comb_stride;
  // Gathered K (gk_start set, block table required): batch entry b sums over
  // the blocks q = gk_bl[4p..4p+3], p in [gk_start[b], gk_start[b+1]), each
  // a K0-long stretch of the contraction whose A and B start at A + cA.q and
  // B + cB.q (the k strides are sAk0, sBk0); C starts at C + cC.bl[4b..4b+3].
  // K is K0 times the largest count.  Entries thus reduce over blocks that
  // share an output without atomics.
  const int* gk_start;
  const int* gk_bl;
  // Column segments (ncs in 1..4, block table required, A read k-fast, atomic
  // accumulation; K0 with sAk1 splits A's k only, the segments' B read the
  // flattened k): columns [16s, 16s + cs[s].n) of
  // the product belong to segment s, which has its own B operand, output and
  // scale,
  //   C_s[m][c] += alpha_s * sum_k A[m][k] B_s[k][c],
  //   B_s[k][c] = cs[s].B[cB_s.(I,J,K,n) + k*sBk + c*sBn],
  //   C_s[m][c] at cs[s].C[cC_s.(I,J,K,n) + m*sCm + c*sCn],
  // so products that share their A operand read it once.  N, the plain B/C
  // fields and alpha are then unused.
  // With tB set (n <= 15), column 15 of the group is a tail column of its own:
  //   C_t[m] += talpha * sum_k A[m][k] tB[tcB.(I,J,K,n) + k*tsBk]  at tC[tcC.(I,J,K,n) + m*tsCm].
  struct ColSeg {
    int n;  // columns, 1..16
    const cplx* B;
    int64_t cB[4], sBk, sBn;
    cplx* C;
    int64_t cC[4], sCm, sCn;
    cplx alpha;
    const cplx* tB;
    int64_t tcB[4], tsBk;
    cplx* tC;
    int64_t tcC[4], tsCm;
    cplx talpha;
  };
  int ncs;
  ColSeg cs[4];
};
void gemm(const GemmDesc& d, hipStream_t s);

// Autotuner of the products' K split.  While tuning, gemm() launches a product
// whose grid is small enough for splitting K to matter once per feasible split
// (powers of two between the accumulation limits and chunks of 64), times each
// with HIP events and keeps the fastest for that product's descriptor (shapes,
// strides, operand modes, precision); afterwards gemm() takes the kept split
// for a descriptor it has seen and its heuristic otherwise.  Tuning launches a
// product several times, so it is only done where repeating a product does no
// harm (the evaluation on the zero state at context set-up).
struct Tuner;
struct TuneRecord {
  int M, N, K, batch, heuristic, chosen;
  float heuristic_ms, chosen_ms;
};
Tuner* tuner_new();
// the tuned products (up to cap into out); returns how many there are
int tuner_records(const Tuner* t, TuneRecord* out, int cap);
void tuner_delete(Tuner* t);
void tuner_set_tuning(Tuner* t, bool on);
void tuner_clear(Tuner* t);
// products tuned, and how many of them run with a split other than the heuristic's
void tuner_counts(const Tuner* t, int& sites, int& changed);
// The tuner gemm() consults on this thread while the scope lives (null: none).
struct TunerScope {
  explicit TunerScope(Tuner* t);
  ~TunerScope();
  Tuner* prev;
};

// Strided elementwise: Y[idx] += alpha * X[idx] over an nd-dim box (nd <= 8).
struct AxpyDesc {
  int nd;
  int64_t shape[8];
  const cplx* X;
  int64_t sx[8];
  cplx* Y;
  int64_t sy[8];
  cplx alpha;
};
void axpy_strided(const AxpyDesc& d, hipStream_t s);

void fill(cplx* p, int64_t n, cplx val, hipStream_t s);
void fill_int(int* p, int64_t n, int val, hipStream_t s);
// Propagation state on the device, so that one RK4 step is the same work every
// time (a captured graph replays it): pst[0] = step within the current chunk,
// pst[1] = first step of the chunk, pst[2] = first diverged step + 1 (0: none).
enum { PST_STEP = 0, PST_BASE = 1, PST_FLAG = 2, PST_N = 4 };
// RK4 update guarded against divergence: cand = y + alpha * a; if an element of
// cand is not finite, pst[PST_FLAG] becomes (pst[PST_BASE] + pst[PST_STEP]) + 1
// unless it is already set; then y = cand unless the flag is set.  Once a step
// diverges, y keeps the last finite state for the rest of the propagation.
// cand must not alias y or a.
void guarded_update(cplx* y, const cplx* a, cplx alpha, cplx* cand, int64_t n, int* pst, hipStream_t s);
// h = h0 - sum_x E_x mu^x (n*n elements), with E read from the device (Edev, 3
// doubles) or, when Edev is null, from ex, ey, ez.
void build_h(cplx* h, const cplx* h0, const cplx* mu, int64_t nn, const double* Edev, const double* Ehost,
             hipStream_t s);
// The four RK4 stage fields of the current step from a field table of samples
// E(k dt/2) (3 doubles each) indexed from the chunk's start: estage[0..2] = E[2c],
// [3..5] = [6..8] = E[2c + 1], [9..11] = E[2c + 2], c = pst[PST_STEP].
void stage_fields(const double* table, const int* pst, double* estage, hipStream_t s);
// mus[3 c + x] = m3[x], c = pst[PST_STEP].
void store_dipole(cplx* mus, const cplx* m3, const int* pst, hipStream_t s);
// pst[PST_STEP] += 1, or pst[PST_STEP] = 0 and pst[PST_BASE] = base (reset).
void advance_step(int* pst, hipStream_t s);
void reset_step(int* pst, int base, hipStream_t s);
// dst[0..n) = src[0..n) on the device (non-overlapping).  A kernel on the
// stream, not a DMA-engine copy, so it orders with the kernels around it
// without an engine switch.
void copy(cplx* dst, const cplx* src, int64_t n, hipStream_t s);

}  // namespace rtcc3
