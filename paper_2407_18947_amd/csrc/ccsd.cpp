// CCSD part of the RT-CC3 right-hand side.
//
// The T side is the closed-shell T1-transformed CCSD residual (expansion
// coefficients of exp(-T2) H~ exp(T2)|0> in {E_ai|0>, 1/2 E_ai E_bj|0>}).  The
// Lambda side is the derivative of the Lagrangian
//   L = E + sum l1.Omega1 + 1/2 sum l2.Omega2
// with respect to t1 and t2 (Euler-Lagrange equations of the CC3 Lagrangian,
// arXiv 2407.18947, Appendix A), taken by a reverse sweep over the recorded
// contractions; the same sweep gives dL/dh~, the one-electron density in the
// T1-transformed frame.
#include "ccsd.h"

#include <cstring>

namespace rtcc3 {

namespace {
constexpr cplx ONE{1.0, 0.0};
inline cplx R(double x) { return cplx{x, 0.0}; }
}  // namespace

CCSDResult ccsd_evaluate(Engine& e, const Dims& d, const cplx* y, const View& h, const View& B, const View& I,
                         const View& ones_o, bool want_grad) {
  CCSDResult r = ccsd_forward(e, d, y, h, B, I, ones_o, want_grad);
  ccsd_residual(e, d, r);
  if (want_grad) ccsd_backward(e, d, y, ones_o, r);
  return r;
}

namespace {
View fresh_view(Engine& e, const char* name, std::vector<int64_t> shape) {
  View t = e.tensor(name, shape);
  e.zero(t);
  e.set_requires_grad(t.buf, false);
  return t;
}
View block_of(const View& x, int64_t o, int64_t n, char a, char b) {
  const int64_t l0 = a == 'o' ? 0 : o, h0 = a == 'o' ? o : n, l1 = b == 'o' ? 0 : o, h1 = b == 'o' ? o : n;
  return Engine::slice(Engine::slice(x, x.nd - 2, l0, h0), x.nd - 1, l1, h1);
}
}  // namespace

CCSDResult ccsd_forward(Engine& e, const Dims& d, const cplx* y, const View& h, const View& B, const View& I,
                        const View& ones_o, bool want_grad) {
  const int64_t o = d.o, v = d.v, n = d.n, na = d.naux;
  const int64_t ov = o * v, oovv = o * o * v * v;
  CCSDResult r;

  // amplitudes: copies of the state's t1, t2 into tracked buffers
  View t1 = e.tensor("t1", {o, v});
  View t2 = e.tensor("t2", {o, o, v, v});
  e.copy(t1.p, y, ov);
  e.copy(t2.p, y + ov, oovv);
  e.set_requires_grad(t1.buf, want_grad);
  e.set_requires_grad(t2.buf, want_grad);
  if (want_grad) e.tape_begin();

  auto fresh = [&](const char* name, std::vector<int64_t> shape) { return fresh_view(e, name, shape); };
  auto blk = [&](const View& x, char a, char b) { return block_of(x, o, n, a, b); };

  // ---- T1 transformation: X = 1 - T, Y = 1 + T with T[a,i] = t_i^a
  View Tm = fresh("Tm", {n, n});
  e.axpy(ONE, Engine::permute(t1, {1, 0}), blk(Tm, 'v', 'o'));
  View X = fresh("Xm", {n, n});
  e.axpy(ONE, I, X);
  e.axpy(R(-1), Tm, X);
  View Y = fresh("Ym", {n, n});
  e.axpy(ONE, I, Y);
  e.axpy(ONE, Tm, Y);
  View hX = fresh("hX", {n, n});
  e.einsum("pr,rq->pq", ONE, X, h, hX);
  View ht = fresh("ht", {n, n});
  e.einsum("pr,rq->pq", ONE, hX, Y, ht);
  View BY = fresh("BY", {na, n, n});
  e.einsum("Prs,sq->Prq", ONE, B, Y, BY);
  View Bt = fresh("Bt", {na, n, n});
  e.einsum("pr,Prq->Ppq", ONE, X, BY, Bt);

  // ---- Fock matrix of the transformed Hamiltonian: F = h~ + sum_k [2 (pq|kk)~ - (pk|kq)~]
  View Bd = fresh("Bd", {na});
  e.einsum("Pk,k->P", ONE, Engine::diag(blk(Bt, 'o', 'o'), 1, 2), ones_o, Bd);
  View F = fresh("F", {n, n});
  e.axpy(ONE, ht, F);
  e.einsum("Ppq,P->pq", R(2), Bt, Bd, F);
  e.einsum("Ppk,Pkq->pq", R(-1), Engine::slice(Bt, 2, 0, o), Engine::slice(Bt, 1, 0, o), F);

  // ---- (ia|jb), invariant under the T1 transformation, for L
  auto gblock = [&](const char* name, const View& BB, const char* s) {
    auto ext = [&](char c) { return c == 'o' ? o : v; };
    View g = fresh(name, {ext(s[0]), ext(s[1]), ext(s[2]), ext(s[3])});
    e.einsum("Ppq,Prs->pqrs", ONE, blk(BB, s[0], s[1]), blk(BB, s[2], s[3]), g);
    return g;
  };
  View g_ovov = gblock("g_ovov", B, "ovov");  // invariant under the T1 transformation

  View u = fresh("u", {o, o, v, v});  // u_ij^ab = 2 t_ij^ab - t_ij^ba
  e.axpy(R(2), t2, u);
  e.axpy(R(-1), Engine::permute(t2, {0, 1, 3, 2}), u);
  View Lov = fresh("Lov", {o, v, o, v});  // L_iajb = 2(ia|jb) - (ib|ja)
  e.axpy(R(2), g_ovov, Lov);
  e.axpy(R(-1), Engine::permute(g_ovov, {0, 3, 2, 1}), Lov);

  r.Bt = Bt;
  r.F = F;
  r.X = X;
  r.Y = Y;
  if (want_grad) e.tape_end();  // paused: the residual continues this tape
  return r;
}

void ccsd_residual(Engine& e, const Dims& d, CCSDResult& r) {
  const int64_t o = d.o, v = d.v, n = d.n;
  const bool want_grad = e.requires_grad(e.tensor("t1", {o, v}).buf);
  if (want_grad) e.tape_resume();
  auto fresh = [&](const char* name, std::vector<int64_t> shape) { return fresh_view(e, name, shape); };
  auto blk = [&](const View& x, char a, char b) { return block_of(x, o, n, a, b); };
  const View t2 = e.tensor("t2", {o, o, v, v}), u = e.tensor("u", {o, o, v, v}), Lov = e.tensor("Lov", {o, v, o, v});
  const View g_ovov = e.tensor("g_ovov", {o, v, o, v});
  const View Bt = r.Bt, F = r.F;
  const View Foo = blk(F, 'o', 'o'), Fov = blk(F, 'o', 'v'), Fvo = blk(F, 'v', 'o'), Fvv = blk(F, 'v', 'v');
  // ---- transformed Mulliken blocks (pq|rs)~
  auto gblock = [&](const char* name, const View& BB, const char* s) {
    auto ext = [&](char c) { return c == 'o' ? o : v; };
    View g = fresh(name, {ext(s[0]), ext(s[1]), ext(s[2]), ext(s[3])});
    e.einsum("Ppq,Prs->pqrs", ONE, blk(BB, s[0], s[1]), blk(BB, s[2], s[3]), g);
    return g;
  };
  View g_vvov = gblock("g_vvov", Bt, "vvov");
  View g_ooov = gblock("g_ooov", Bt, "ooov");
  View g_vovo = gblock("g_vovo", Bt, "vovo");
  View g_vvvv = gblock("g_vvvv", Bt, "vvvv");
  View g_oooo = gblock("g_oooo", Bt, "oooo");
  View g_oovv = gblock("g_oovv", Bt, "oovv");
  View g_voov = gblock("g_voov", Bt, "voov");
  View g_vvoo = gblock("g_vvoo", Bt, "vvoo");

  // ---- singles
  View R1 = fresh("R1", {o, v});
  e.einsum("kicd,adkc->ia", ONE, u, g_vvov, R1);
  e.einsum("klac,kilc->ia", R(-1), u, g_ooov, R1);
  e.einsum("ikac,kc->ia", ONE, u, Fov, R1);
  e.axpy(ONE, Engine::permute(Fvo, {1, 0}), R1);

  // ---- doubles
  View R2 = fresh("R2", {o, o, v, v});
  e.axpy(ONE, Engine::permute(g_vovo, {1, 3, 0, 2}), R2);
  e.einsum("ijcd,acbd->ijab", ONE, t2, g_vvvv, R2);
  View Xkl = fresh("Xkl", {o, o, o, o});
  e.axpy(ONE, Engine::permute(g_oooo, {0, 2, 1, 3}), Xkl);
  e.einsum("ijcd,kcld->klij", ONE, t2, g_ovov, Xkl);
  e.einsum("klab,klij->ijab", ONE, t2, Xkl, R2);

  View Cx = fresh("Cx", {o, o, v, v});  // terms symmetrised with P_ij^ab
  View Yk = fresh("Yk", {o, o, v, v});
  e.axpy(ONE, g_oovv, Yk);
  e.einsum("liad,kdlc->kiac", R(-0.5), t2, g_ovov, Yk);
  e.einsum("kjbc,kiac->ijab", R(-0.5), t2, Yk, Cx);
  e.einsum("kibc,kjac->ijab", R(-1), t2, Yk, Cx);
  View Zd = fresh("Zd", {v, o, o, v});
  e.axpy(R(2), g_voov, Zd);
  e.axpy(R(-1), Engine::permute(g_vvoo, {0, 3, 2, 1}), Zd);
  e.einsum("ilad,ldkc->aikc", R(0.5), u, Lov, Zd);
  e.einsum("jkbc,aikc->ijab", R(0.5), u, Zd, Cx);
  View Wvv = fresh("Wvv", {v, v});
  e.axpy(ONE, Fvv, Wvv);
  e.einsum("klbd,ldkc->bc", R(-1), u, g_ovov, Wvv);
  e.einsum("ijac,bc->ijab", ONE, t2, Wvv, Cx);
  View Woo = fresh("Woo", {o, o});
  e.axpy(ONE, Foo, Woo);
  e.einsum("ljcd,kdlc->kj", ONE, u, g_ovov, Woo);
  e.einsum("ikab,kj->ijab", R(-1), t2, Woo, Cx);
  e.axpy(ONE, Cx, R2);
  e.axpy(ONE, Engine::permute(Cx, {1, 0, 3, 2}), R2);

  r.R1 = R1;
  r.R2 = R2;
  if (want_grad) e.tape_end();
}

void ccsd_backward(Engine& e, const Dims& d, const cplx* y, const View& ones_o, CCSDResult& r) {
  const int64_t o = d.o, v = d.v, n = d.n;
  const int64_t ov = o * v, oovv = o * o * v * v;
  auto blk = [&](const View& x, char a, char b) { return block_of(x, o, n, a, b); };
  const View t1 = e.tensor("t1", {o, v}), t2 = e.tensor("t2", {o, o, v, v});
  const View ht = e.tensor("ht", {n, n}), Lov = e.tensor("Lov", {o, v, o, v});

  // ---- reverse sweep.  Seeds: dL/dOmega1 = l1, dL/dOmega2 = 1/2 l2, and the
  // energy E = sum_i (h~_ii + F_ii) + sum_ijab t_ij^ab L_iajb contributes
  // dE/dh~_ii = dE/dF_ii = 1 (occupied i) and dE/dt2 = L.
  e.zero_grads();
  View gR1 = e.grad(r.R1), gR2 = e.grad(r.R2);
  e.copy(gR1.p, y + ov + oovv, ov);
  View l2 = Engine::raw(const_cast<cplx*>(y) + 2 * ov + oovv, {o, o, v, v});
  e.axpy(R(0.5), l2, gR2);
  e.axpy(ONE, ones_o, Engine::diag(blk(e.grad(r.F), 'o', 'o'), 0, 1));
  e.axpy(ONE, ones_o, Engine::diag(blk(e.grad(ht), 'o', 'o'), 0, 1));
  e.axpy(ONE, Engine::permute(Lov, {0, 2, 1, 3}), e.grad(t2));
  e.backward();
  r.G1 = e.grad(t1);
  r.G2 = e.grad(t2);
  r.Dt = e.grad(ht);
}

cplx ccsd_energy(Engine& e, const Dims& d, const CCSDResult& r) {
  const int64_t o = d.o, v = d.v, n = d.n;
  View Es = e.tensor("Eval", {});
  e.zero(Es);
  View ht = e.tensor("ht", {n, n});
  View ones = e.tensor("ones_o", {o});
  View t2 = e.tensor("t2", {o, o, v, v});
  View Lov = e.tensor("Lov", {o, v, o, v});
  auto oo = [&](const View& x) { return Engine::slice(Engine::slice(x, 0, 0, o), 1, 0, o); };
  e.einsum("i,i->", ONE, Engine::diag(oo(ht), 0, 1), ones, Es);
  e.einsum("i,i->", ONE, Engine::diag(oo(r.F), 0, 1), ones, Es);
  e.einsum("ijab,iajb->", ONE, t2, Lov, Es);
  cplx out;
  RTCC3_HIP(hipMemcpyAsync(&out, Es.p, sizeof(cplx), hipMemcpyDeviceToHost, e.stream));
  RTCC3_HIP(hipStreamSynchronize(e.stream));
  return out;
}

}  // namespace rtcc3
