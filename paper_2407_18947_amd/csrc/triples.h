// Approximate triples of CC3 evaluated one occupied triple (i,j,k) at a time.
#pragma once

#include <functional>
#include <vector>

#include "ccsd.h"
#include "engine.h"

namespace rtcc3 {

struct TriplesOut {
  View X1, X2, Y1, Y2;  // contributions to the T and Lambda residuals
  View Dij, Dab, Dia;   // triples part of the T1-frame density (when requested)
};

// The blocks the right-hand-side contractions run over (all blocks, or the
// owned ones of a pair window) grouped by one of their occupied indices, for
// products that reduce over the blocks sharing an output (GemmDesc::gk_*).
struct Groups {
  std::vector<int> key;    // [ng][4]: the shared index at its position, zeros elsewhere
  std::vector<int> start;  // [ng + 1]: group g is bl entries [start[g], start[g+1])
  std::vector<int> bl;     // [*][4]: (I, J, K, n) in group order
  int max = 0;             // largest group
  int* d_key = nullptr;
  int* d_start = nullptr;
  int* d_bl = nullptr;
};

// A window: a set of ordered occupied triples that is closed under permutation,
// so every block's P_ijk^abc partners are in it.  The contraction set (all
// blocks, or the owned ones) is a union of whole permutation orbits as well.
struct Window {
  int nw = 0;                 // ordered blocks
  std::vector<int> bl;        // [nw][4]: I, J, K, n (host copy)
  std::vector<int> part;      // [nw][6]: window indices of (ijk),(jik),(ikj),(kji),(kij),(jki)
  std::vector<int> owned;     // [*][4]: blocks whose density terms this window accumulates
  std::vector<int> canon;     // [*][4]: I <= J <= K and the slot of that ordering, one per distinct triple
  std::vector<int> slabs;     // density windows: [*][4] = (0, 0, 0, slot of block (0,l,k)); the o blocks
                              // (i,l,k) of a slab occupy consecutive slots in i
  Groups gJ, gK;              // contraction blocks grouped by J and by K
  std::vector<int> orb;       // bl, and owned, with the orderings of each occupied triple consecutive
  std::vector<int> orb_owned;
  // bl sorted by (K, J, I) and by (K, I, J), and owned by (K, I, J), for the
  // build products: neighbouring entries then share their largest operand
  // blocks, which stay in the L2 cache for them
  std::vector<int> bk_t3, bk_l3, bk_own;
  int* d_bl = nullptr;
  int* d_part = nullptr;
  int* d_owned = nullptr;
  int* d_canon = nullptr;
  int* d_slabs = nullptr;
  int* d_orb = nullptr;
  int* d_orb_owned = nullptr;
  int* d_bk_t3 = nullptr;
  int* d_bk_l3 = nullptr;
  int* d_bk_own = nullptr;
};

class Triples {
 public:
  Triples(Engine& e, const Dims& d, const std::vector<double>& eps, int precision);
  ~Triples();
  // Run all windows.  want_density: also the triples density terms; the pass
  // then runs over the density windows: one window of every block when all o^3
  // fit, else pair windows that hold, for occupied pairs (l,k), the slabs of
  // blocks (i,l,k) of every i and evaluate the right-hand side for the blocks
  // each window owns.
  // beside (optional) is called once, after the first window's lambda3 build
  // has been enqueued, with an event recorded after that build: it may enqueue
  // independent work on another stream that waits for the event (so the work
  // runs beside the contractions rather than the builds) and returns an event
  // recorded after it, which side_done() returns until the next run; run()
  // does not wait for it.  ready (optional): an event after which the integral
  // blocks of the CCSD residual that the final contractions read are complete.
  typedef std::function<hipEvent_t(hipEvent_t)> Beside;
  TriplesOut run(Engine& e, const Dims& d, const CCSDResult& r, const cplx* y, bool want_density,
                 const Beside& beside = nullptr, hipEvent_t ready = nullptr);
  hipEvent_t side_done() const { return side_done_; }
  void set_precision(int p) { prec_ = p; }
  // All work on the caller's stream, one kernel after another (for timing
  // kernels alone); the default runs the lambda3 side on a second stream.
  void set_single_stream(bool on) { single_ = on; }
  // Cap the blocks per window (0: sized from free device memory) and rebuild
  // the windows; the window buffers are released and reallocated on use.
  void set_window_blocks(Engine& e, int n);
  void reset_timing() {
    fold_timing();
    ms_ = 0;
    launches_ = 0;
    build_ms_ = 0;
    build_launches_ = 0;
    build_flop_ = 0;
  }
  // Record timing events (default); off while a graph is captured, whose
  // replays are timed as a whole by the caller.
  void set_timing(bool on) { timing_on_ = on; }
  // Wait for the timing events recorded so far and add up their intervals
  // (call after the caller's stream has been synchronised; also done by run()
  // itself when an event pool is full).
  void fold_timing();
  void timing(double& ms, double& launches) const {
    ms = ms_;
    launches = (double)launches_;
  }
  // The segmented store-mode products (the t3 and lambda3 builds and the Y1 S
  // intermediate, one kernel): event-timed milliseconds, launches and
  // algorithmic flops (8 per complex multiply-add).
  void build_timing(double& ms, double& launches, double& flop) const {
    ms = build_ms_;
    launches = (double)build_launches_;
    flop = build_flop_;
  }

 private:
  Dims d_;
  int prec_;
  bool single_ = false;
  double* eps_ = nullptr;  // device
  std::vector<Window> rhs_windows_, den_windows_;
  int max_nw_ = 0;
  int wcap_ = 0;  // blocks per window requested by the caller (0: from the memory budget)
  double ms_ = 0;
  long launches_ = 0;
  double build_ms_ = 0, build_flop_ = 0;
  long build_launches_ = 0;
  // Timing events, all created with the engine: pairs around each run (rev_)
  // and around each launch of the build products (bev_), folded into the
  // totals by fold_timing() so that no run waits for the device.
  std::vector<hipEvent_t> rev_, bev_;
  int nrev_ = 0;
  bool timing_on_ = true;
  // A window's lambda3 side (build, symmetrisation, the contractions that read
  // lambda3 only) runs on a second stream beside the t3 side; ev_fork_ /
  // ev_l_ / ev_join_ order the two.
  hipStream_t s2_ = nullptr;
  hipEvent_t ev_fork_ = nullptr, ev_l_ = nullptr, ev_join_ = nullptr;
  hipEvent_t ev_t_ = nullptr;    // t3 blocks ready (D_ij on the lambda3 side reads them)
  hipEvent_t ev_t3b_ = nullptr;  // after the t3 build: both builds are bound by the
                                 // matrix cores, so the lambda3 build follows it
  hipEvent_t ev_l3b_ = nullptr;  // after the lambda3 build: the t3 side's products wait for it
                                 // and only the t3 symmetrisation runs beside it
  int nbev_ = 0;                 // events recorded since the last fold
  const Beside* beside_ = nullptr;  // pending side work of the current run
  hipEvent_t side_done_ = nullptr;
  void build_event(hipStream_t s);

  void build_windows();
  void upload(Window& w);
  void free_windows();
  void blocks(Engine& e, const CCSDResult& r);
  void window_pass(Engine& e, const Window& w, const cplx* y, bool rhs_terms, bool density_terms);
};

}  // namespace rtcc3
