// T1 transformation and the CCSD part of the RT-CC3 right-hand side on the
// contraction engine (forward program + reverse sweep).
#pragma once

#include "engine.h"

namespace rtcc3 {

struct Dims {
  int o, v, n, naux;
};

// Views produced by one evaluation (valid until the next call).
struct CCSDResult {
  View Bt;   // [naux, n, n] T1-transformed DF factors
  View F;    // [n, n] T1-transformed Fock matrix
  View X, Y; // [n, n] (1 - T), (1 + T)
  View R1, R2;          // Omega_1 [o,v], Omega_2 [o,o,v,v]
  View G1, G2;          // dL/dt1, dL/dt2 (CCSD part of the Lagrangian)
  View Dt;              // dL/dh~ (CCSD part of the T1-frame density) [n, n]
};

// Evaluate with t1, t2 and lambda seeds taken from the state vector y (device).
// h: bare one-electron operator including the field [n,n] (complex view).
// want_grad: also the reverse sweep (G1, G2, Dt).
CCSDResult ccsd_evaluate(Engine& e, const Dims& d, const cplx* y, const View& h, const View& B,
                         const View& I, const View& ones_o, bool want_grad);
// The three parts of ccsd_evaluate, in this order on one engine tape:
// ccsd_forward - T1 transformation, f~, L and u (what the triples read);
// ccsd_residual - the transformed (pq|rs)~ blocks and Omega1, Omega2 (r.R1, r.R2);
// ccsd_backward - the reverse sweep (r.G1, r.G2, r.Dt).
// The last two read only engine buffers of the forward part and y, and write
// their own, so they may run on another stream (the engine's stream switched)
// while other work reads the forward part's buffers; the tape is paused
// between the forward part and the residual.
CCSDResult ccsd_forward(Engine& e, const Dims& d, const cplx* y, const View& h, const View& B, const View& I,
                        const View& ones_o, bool want_grad = true);
void ccsd_residual(Engine& e, const Dims& d, CCSDResult& r);
void ccsd_backward(Engine& e, const Dims& d, const cplx* y, const View& ones_o, CCSDResult& r);

// Energy of the CCSD part (for tests): E = sum_i (h~_ii + F~_ii) + sum t2 L.
cplx ccsd_energy(Engine& e, const Dims& d, const CCSDResult& r);

}  // namespace rtcc3
