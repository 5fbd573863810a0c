// Launchers of the triples engine's element-wise kernels (triples_kernels.hip).
// bl: block table, 4 ints per entry (I, J, K, n) with n the block's slot in the
// window buffers; part: 6 window slots per entry (see Window in triples.h).
#pragma once

#include "common.h"

namespace rtcc3 {

// Inputs of the lambda3 bracket terms that carry no summation index.
struct LamElem {
  const cplx* Lov = nullptr;  // L_iajb = 2(ia|jb)~ - (ib|ja)~, [o][v][o][v]
  const cplx* F = nullptr;    // dressed Fock, [n][n]
  const cplx* l1 = nullptr;   // [o][v]
  const cplx* l2 = nullptr;   // [o][o][v][v]
};
// Symmetrise and divide, in place, for the canonical triples of a window
// (canon: 4 ints per entry, I <= J <= K and the slot of that ordering): every
// ordering's block of W is replaced by the symmetrised, divided result.
// le (may be null): add the lambda3 bracket terms without a summation index to
// every source element first; le2 (may be null): add them for a second set of
// inputs too.  A null input of a set reads as zero.  Blocks are [v][v][vp]:
// vp >= v is the row stride of the innermost index.
void launch_sym_cube(cplx* W, const int* canon, int ncanon, const int* part, const double* eps, int o, int v, int vp,
                     const LamElem* le, const LamElem* le2, hipStream_t s);
// D[i][j] += alpha * sum_s sum_k A[(slot_s + i)*K + k] B[(slot_s + j)*K + k] for
// i, j < o <= 16, slot_s = slabs[4 s + 3] (the slab's o blocks are consecutive
// slots of K elements each).  D is [o][o], accumulated with atomics.
void launch_gram(const cplx* A, const cplx* B, const int* slabs, int nslab, int o, int64_t K, cplx alpha, cplx* D,
                 hipStream_t s);
// X1, the f~ term of X2 and Z (terms 3 and 4 of Y1) by one sweep per block
// (blocks [v][v][vp] as above).
void launch_small_t3(const cplx* T, const int* bl, int nb, const cplx* Lov, const cplx* F, const cplx* l2, cplx* X1,
                     cplx* X2p, cplx* Z, int o, int v, int vp, int flags, hipStream_t s);

}  // namespace rtcc3
