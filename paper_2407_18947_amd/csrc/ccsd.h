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
// The two halves of ccsd_evaluate(..., true): the forward program (recorded),
// and the reverse sweep that fills r.G1, r.G2, r.Dt.  The sweep reads only the
// engine buffers of the forward program and y, and writes gradient buffers, so
// it may run on another stream while other work reads those buffers.
CCSDResult ccsd_forward(Engine& e, const Dims& d, const cplx* y, const View& h, const View& B, const View& I,
                        const View& ones_o);
void ccsd_backward(Engine& e, const Dims& d, const cplx* y, const View& ones_o, CCSDResult& r);

// Energy of the CCSD part (for tests): E = sum_i (h~_ii + F~_ii) + sum t2 L.
cplx ccsd_energy(Engine& e, const Dims& d, const CCSDResult& r);

}  // namespace rtcc3
