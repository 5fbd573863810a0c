// Launchers of the triples engine's element-wise kernels (triples_kernels.hip).
// bl: block table, 4 ints per entry (I, J, K, n) with n the block's slot in the
// window buffers; part: 6 window slots per entry (see Window in triples.h).
#pragma once

#include "common.h"

namespace rtcc3 {

void launch_sym_div(const cplx* W, cplx* T, const int* part, const int* bl, const double* eps, int o, int v, int nb,
                    hipStream_t s);
// Symmetrise and divide for the canonical triples of a window (canon: 4 ints
// per entry, I <= J <= K and the slot of that ordering); writes all orderings.
void launch_sym_cube(const cplx* W, cplx* T, const int* canon, int ncanon, const int* part, const double* eps, int o,
                     int v, hipStream_t s);
void launch_lam_elem(cplx* W, const int* bl, const cplx* Lov, const cplx* F, const cplx* l1, const cplx* l2, int o,
                     int v, int nb, hipStream_t s);
void launch_comb(const cplx* T, cplx* Z, const int* bl, int v, int nb, int mode, hipStream_t s);
void launch_small_t3(const cplx* T, const int* bl, int nb, const cplx* Lov, const cplx* F, const cplx* l2, cplx* X1,
                     cplx* X2p, cplx* Z, int o, int v, int flags, hipStream_t s);

}  // namespace rtcc3
