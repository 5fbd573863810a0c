#include "engine.h"

#include <algorithm>
#include <cstring>

namespace rtcc3 {

Engine::~Engine() {
  for (auto& b : bufs_)
    for (cplx* q : {b.p, b.g, b.tp, b.tg})
      if (q) (void)hipFree(q);
  for (auto& sc : scratch_)
    if (sc.p) (void)hipFree(sc.p);
}

cplx* Engine::alloc_twin(int64_t n) {
  cplx* q = nullptr;
  if (n <= 0) return q;
  if (sealed_) throw Error(-4, "engine: twin allocated after the context was set up");
  hipError_t e = hipMalloc(&q, sizeof(cplx) * n);
  if (e != hipSuccess) throw Error(-2, "engine: out of device memory for a tangent twin");
  RTCC3_HIP(hipMemsetAsync(q, 0, sizeof(cplx) * n, stream));
  return q;
}

void Engine::enable_twins() {
  if (twins_) return;
  for (auto& b : bufs_) {
    if (b.p && !b.tp) b.tp = alloc_twin(b.n);
    if (b.g && !b.tg) b.tg = alloc_twin(b.n);
    b.tp_nz = b.tg_nz = false;
  }
  twins_ = true;
}

const Engine::Range* Engine::find(const cplx* p, int64_t* off) const {
  auto it = ranges_.upper_bound(p);
  if (it == ranges_.begin()) return nullptr;
  --it;
  const int64_t d = p - it->first;
  if (d < 0 || d >= it->second.n) return nullptr;
  *off = d;
  return &it->second;
}

const cplx* Engine::twin(const cplx* p) const {
  int64_t off = 0;
  const Range* r = find(p, &off);
  if (!r) return nullptr;
  const Buf& b = bufs_[r->buf];
  if (r->kind == 0) return b.tp_nz ? b.tp + off : nullptr;
  return b.tg_nz ? b.tg + off : nullptr;
}

cplx* Engine::twin_out(const cplx* p) {
  int64_t off = 0;
  const Range* r = find(p, &off);
  RTCC3_CHECK(r != nullptr, "engine: derivative written to memory outside the engine's buffers");
  Buf& b = bufs_[r->buf];
  cplx* t = r->kind == 0 ? b.tp : b.tg;
  RTCC3_CHECK(t != nullptr, "engine: buffer '" + b.name + "' has no tangent twin");
  (r->kind == 0 ? b.tp_nz : b.tg_nz) = true;
  return t + off;
}

void Engine::copy(cplx* dst, const cplx* src, int64_t n) {
  rtcc3::copy(dst, src, n, stream);
  if (!tangent_) return;
  const cplx* st = twin(src);
  if (st) {
    rtcc3::copy(twin_out(dst), st, n, stream);
    return;
  }
  int64_t off = 0;
  const Range* r = find(dst, &off);
  RTCC3_CHECK(r != nullptr, "engine: copy into memory outside the engine's buffers");
  Buf& b = bufs_[r->buf];
  const bool nz = r->kind == 0 ? b.tp_nz : b.tg_nz;
  if (nz) fill((r->kind == 0 ? b.tp : b.tg) + off, n, cplx{0, 0}, stream);
}

int Engine::buffer(const std::string& name, int64_t n) {
  auto it = names_.find(name);
  if (it != names_.end()) {
    RTCC3_CHECK(bufs_[it->second].n == n, "engine: buffer '" + name + "' requested with a different size");
    return it->second;
  }
  if (sealed_) throw Error(-4, "engine: buffer '" + name + "' requested after the context was set up");
  Buf b;
  b.name = name;
  b.n = n;
  if (n > 0) {
    hipError_t e = hipMalloc(&b.p, sizeof(cplx) * n);
    if (e != hipSuccess) throw Error(-2, "engine: out of device memory for '" + name + "'");
    RTCC3_HIP(hipMemsetAsync(b.p, 0, sizeof(cplx) * n, stream));
    if (twins_) b.tp = alloc_twin(n);
  }
  bufs_.push_back(b);
  const int id = (int)bufs_.size() - 1;
  names_[name] = id;
  if (b.p) ranges_[b.p] = Range{n, id, 0};
  return id;
}

void Engine::release(const std::string& name) {
  auto it = names_.find(name);
  if (it == names_.end()) return;
  RTCC3_HIP(hipStreamSynchronize(stream));
  Buf& b = bufs_[it->second];
  if (b.p) ranges_.erase(b.p);
  if (b.g) ranges_.erase(b.g);
  for (cplx* q : {b.p, b.g, b.tp, b.tg})
    if (q) RTCC3_HIP(hipFree(q));
  b.p = b.g = b.tp = b.tg = nullptr;
  b.tp_nz = b.tg_nz = false;
  b.n = 0;
  b.rg = false;
  names_.erase(it);
}

View Engine::tensor_of(int buf, std::vector<int64_t> shape) {
  View v;
  v.nd = (int)shape.size();
  RTCC3_CHECK(v.nd <= 8, "engine: too many dimensions");
  int64_t s = 1;
  for (int k = v.nd - 1; k >= 0; --k) {
    v.sh[k] = shape[k];
    v.st[k] = s;
    s *= shape[k];
  }
  RTCC3_CHECK(s <= bufs_[buf].n, "engine: view larger than its buffer");
  v.p = bufs_[buf].p;
  v.buf = buf;
  v.off = 0;
  return v;
}

View Engine::tensor(const std::string& name, std::vector<int64_t> shape) {
  int64_t n = 1;
  for (auto x : shape) n *= x;
  return tensor_of(buffer(name, n), shape);
}

View Engine::raw(cplx* p, std::vector<int64_t> shape) {
  View v;
  v.nd = (int)shape.size();
  int64_t s = 1;
  for (int k = v.nd - 1; k >= 0; --k) {
    v.sh[k] = shape[k];
    v.st[k] = s;
    s *= shape[k];
  }
  v.p = p;
  return v;
}

void Engine::zero(const View& v) {
  // zero the elements of a view (contiguous fast path, else axpy with -1 of itself is wrong; use fill)
  bool contiguous = true;
  int64_t s = 1;
  for (int k = v.nd - 1; k >= 0; --k) {
    if (v.sh[k] != 1 && v.st[k] != s) contiguous = false;
    s *= v.sh[k];
  }
  RTCC3_CHECK(contiguous, "engine: zero() needs a contiguous view");
  fill(v.p, v.numel(), cplx{0, 0}, stream);
  if (!twins_) return;
  int64_t off = 0;
  const Range* r = find(v.p, &off);
  if (!r) return;
  Buf& b = bufs_[r->buf];
  bool& nz = r->kind == 0 ? b.tp_nz : b.tg_nz;
  if (!nz) return;  // already zero
  fill((r->kind == 0 ? b.tp : b.tg) + off, v.numel(), cplx{0, 0}, stream);
  if (off == 0 && v.numel() == b.n) nz = false;
}

void Engine::zero_buffer(int buf) {
  Buf& b = bufs_[buf];
  fill(b.p, b.n, cplx{0, 0}, stream);
  if (b.tp_nz) fill(b.tp, b.n, cplx{0, 0}, stream);
  b.tp_nz = false;
}

View Engine::slice(View v, int dim, int64_t lo, int64_t hi) {
  RTCC3_CHECK(dim < v.nd && lo >= 0 && hi <= v.sh[dim] && lo <= hi, "engine: bad slice");
  v.p += lo * v.st[dim];
  v.off += lo * v.st[dim];
  v.sh[dim] = hi - lo;
  return v;
}

View Engine::permute(View v, std::vector<int> perm) {
  RTCC3_CHECK((int)perm.size() == v.nd, "engine: bad permutation");
  View w = v;
  for (int d = 0; d < v.nd; ++d) {
    w.sh[d] = v.sh[perm[d]];
    w.st[d] = v.st[perm[d]];
  }
  return w;
}

View Engine::diag(View v, int d0, int d1) {
  RTCC3_CHECK(d0 < d1 && d1 < v.nd && v.sh[d0] == v.sh[d1], "engine: bad diagonal");
  View w;
  w.p = v.p;
  w.buf = v.buf;
  w.off = v.off;
  int k = 0;
  for (int d = 0; d < v.nd; ++d) {
    if (d == d1) continue;
    w.sh[k] = v.sh[d];
    w.st[k] = (d == d0) ? v.st[d0] + v.st[d1] : v.st[d];
    ++k;
  }
  w.nd = k;
  return w;
}

cplx* Engine::scratch(int64_t n) {
  Scratch* sc = nullptr;
  for (auto& x : scratch_)
    if (x.stream == stream) sc = &x;
  if (!sc) {
    if (sealed_) throw Error(-4, "engine: scratch for a new stream after the context was set up");
    scratch_.push_back(Scratch{stream, nullptr, 0});
    sc = &scratch_.back();
  }
  if (n > sc->n) {
    if (sealed_) throw Error(-4, "engine: scratch grown after the context was set up");
    // work on any stream may still read the old scratch
    RTCC3_HIP(hipDeviceSynchronize());
    if (sc->p) RTCC3_HIP(hipFree(sc->p));
    sc->p = nullptr;
    hipError_t e = hipMalloc(&sc->p, sizeof(cplx) * n);
    if (e != hipSuccess) throw Error(-2, "engine: out of device memory for scratch");
    sc->n = n;
  }
  return sc->p;
}

void Engine::set_requires_grad(int buf, bool on) { bufs_[buf].rg = on; }

View Engine::grad(const View& v) {
  RTCC3_CHECK(v.buf >= 0 && bufs_[v.buf].rg, "engine: grad() of a view without gradient");
  Buf& b = bufs_[v.buf];
  if (!b.g) {
    if (sealed_) throw Error(-4, "engine: gradient of '" + b.name + "' requested after the context was set up");
    hipError_t e = hipMalloc(&b.g, sizeof(cplx) * b.n);
    if (e != hipSuccess) throw Error(-2, "engine: out of device memory for a gradient");
    RTCC3_HIP(hipMemsetAsync(b.g, 0, sizeof(cplx) * b.n, stream));
    ranges_[b.g] = Range{b.n, v.buf, 1};
    if (twins_) b.tg = alloc_twin(b.n);
  }
  View g = v;
  g.p = b.g + v.off;
  g.buf = -1;
  return g;
}

void Engine::tape_begin() {
  tape_.clear();
  recording_ = true;
}

void Engine::zero_grads() {
  for (auto& b : bufs_)
    if (b.rg && b.g) {
      fill(b.g, b.n, cplx{0, 0}, stream);
      if (b.tg_nz) fill(b.tg, b.n, cplx{0, 0}, stream);
      b.tg_nz = false;
    }
}

void Engine::axpy(cplx alpha, const View& X, const View& Y) {
  axpy_exec(alpha, X, Y);
  if (tangent_) {
    const cplx* xt = twin(X.p);
    if (xt) {
      View Xt = X, Yt = Y;
      Xt.p = const_cast<cplx*>(xt);
      Yt.p = twin_out(Y.p);
      axpy_exec(alpha, Xt, Yt);
    }
  }
  if (recording_ && requires_grad(X.buf)) {
    if (Y.buf >= 0) bufs_[Y.buf].rg = true;
    tape_.push_back(Op{1, "", alpha, X, View(), Y});
  }
}

void Engine::axpy_exec(cplx alpha, const View& X, const View& Y) {
  RTCC3_CHECK(X.nd == Y.nd, "engine: axpy rank mismatch");
  AxpyDesc d;
  d.nd = X.nd;
  for (int k = 0; k < X.nd; ++k) {
    RTCC3_CHECK(X.sh[k] == Y.sh[k], "engine: axpy shape mismatch");
    d.shape[k] = X.sh[k];
    d.sx[k] = X.st[k];
    d.sy[k] = Y.st[k];
  }
  d.X = X.p;
  d.Y = Y.p;
  d.alpha = alpha;
  axpy_strided(d, stream);
}

void Engine::einsum_dual(const std::string& spec, cplx alpha, const View& A, const View& B, const View& C) {
  // the twins of the inputs are looked up before C's is marked written
  const cplx* at = tangent_ ? twin(A.p) : nullptr;
  const cplx* bt = tangent_ ? twin(B.p) : nullptr;
  einsum_exec(spec, alpha, A, B, C);
  if (!at && !bt) return;
  View Ct = C;
  Ct.p = twin_out(C.p);
  if (at) {
    View At = A;
    At.p = const_cast<cplx*>(at);
    einsum_exec(spec, alpha, At, B, Ct);
  }
  if (bt) {
    View Bt = B;
    Bt.p = const_cast<cplx*>(bt);
    einsum_exec(spec, alpha, A, Bt, Ct);
  }
}

void Engine::einsum(const char* spec, cplx alpha, const View& A, const View& B, const View& C) {
  einsum_dual(spec, alpha, A, B, C);
  if (recording_ && (requires_grad(A.buf) || requires_grad(B.buf))) {
    if (C.buf >= 0) bufs_[C.buf].rg = true;
    tape_.push_back(Op{0, spec, alpha, A, B, C});
  }
}

void Engine::backward() {
  recording_ = false;
  for (auto it = tape_.rbegin(); it != tape_.rend(); ++it) {
    const Op& op = *it;
    if (op.C.buf < 0 || !bufs_[op.C.buf].rg || !bufs_[op.C.buf].g) continue;
    View gC = grad(op.C);
    if (op.kind == 1) {
      if (requires_grad(op.A.buf)) axpy(op.alpha, gC, grad(op.A));
      continue;
    }
    const std::string& s = op.spec;
    const size_t c1 = s.find(','), c2 = s.find("->");
    const std::string sa = s.substr(0, c1), sb = s.substr(c1 + 1, c2 - c1 - 1), sc = s.substr(c2 + 2);
    if (requires_grad(op.A.buf)) einsum_dual(sc + "," + sb + "->" + sa, op.alpha, gC, op.B, grad(op.A));
    if (requires_grad(op.B.buf)) einsum_dual(sa + "," + sc + "->" + sb, op.alpha, op.A, gC, grad(op.B));
  }
}

// ---------------------------------------------------------------------------
// einsum -> one batched GEMM
// ---------------------------------------------------------------------------
namespace {

struct Operand {
  std::string idx;
  const View* v;
  int64_t stride(char c) const {
    size_t p = idx.find(c);
    return p == std::string::npos ? 0 : v->st[p];
  }
};

// Break points (positions inside group g) where the memory layout of x does not
// continue the previous index contiguously; size-1 indices are ignored.
std::vector<int> breaks(const Operand& x, const std::string& g, const std::map<char, int64_t>& ext) {
  std::vector<int> out;
  int prev = -1;
  for (int i = 0; i < (int)g.size(); ++i) {
    if (ext.at(g[i]) == 1) continue;
    if (prev >= 0 && x.stride(g[prev]) != x.stride(g[i]) * ext.at(g[i])) out.push_back(i);
    prev = i;
  }
  return out;
}

// Two-level decomposition of group g at split position sp (elements g[sp..] form
// the inner level).  Returns (inner extent, outer stride, inner stride).
void level_strides(const Operand& x, const std::string& g, int sp, const std::map<char, int64_t>& ext,
                   int64_t& inner, int64_t& s1, int64_t& s0) {
  inner = 1;
  s1 = 0;
  s0 = 0;
  for (int i = sp; i < (int)g.size(); ++i) inner *= ext.at(g[i]);
  int last0 = -1, last1 = -1;
  for (int i = 0; i < (int)g.size(); ++i) {
    if (ext.at(g[i]) == 1) continue;
    if (i >= sp)
      last0 = i;
    else
      last1 = i;
  }
  if (last0 >= 0) s0 = x.stride(g[last0]);
  if (last1 >= 0) s1 = x.stride(g[last1]);
}

int64_t extent(const std::string& g, const std::map<char, int64_t>& ext) {
  int64_t n = 1;
  for (char c : g) n *= ext.at(c);
  return n;
}

}  // namespace

void Engine::einsum_exec(const std::string& spec, cplx alpha, const View& A0, const View& B0, const View& C0) {
  const size_t c1 = spec.find(','), c2 = spec.find("->");
  RTCC3_CHECK(c1 != std::string::npos && c2 != std::string::npos, "einsum: bad spec " + spec);
  std::string sa = spec.substr(0, c1), sb = spec.substr(c1 + 1, c2 - c1 - 1), sc = spec.substr(c2 + 2);
  RTCC3_CHECK((int)sa.size() == A0.nd && (int)sb.size() == B0.nd && (int)sc.size() == C0.nd,
              "einsum: rank mismatch in " + spec);
  std::map<char, int64_t> ext;
  auto add = [&](const std::string& s, const View& v) {
    for (int i = 0; i < (int)s.size(); ++i) {
      auto it = ext.find(s[i]);
      if (it == ext.end())
        ext[s[i]] = v.sh[i];
      else
        RTCC3_CHECK(it->second == v.sh[i], "einsum: extent mismatch for index in " + spec);
    }
  };
  add(sa, A0);
  add(sb, B0);
  add(sc, C0);
  for (auto& kv : ext)
    if (kv.second == 0) return;  // empty contraction or output
  std::string gb, gm, gn, gk;
  for (char c : sc) {
    const bool ina = sa.find(c) != std::string::npos, inb = sb.find(c) != std::string::npos;
    RTCC3_CHECK(ina || inb, "einsum: output index not in inputs: " + spec);
    if (ina && inb)
      gb += c;
    else if (ina)
      gm += c;
    else
      gn += c;
  }
  for (char c : sa)
    if (sc.find(c) == std::string::npos) {
      RTCC3_CHECK(sb.find(c) != std::string::npos, "einsum: index summed in one operand only: " + spec);
      gk += c;
    }
  for (char c : sb)
    if (sc.find(c) == std::string::npos)
      RTCC3_CHECK(sa.find(c) != std::string::npos, "einsum: index summed in one operand only: " + spec);

  View A = A0, B = B0, C = C0;
  Operand oa{sa, &A}, ob{sb, &B}, oc{sc, &C};

  // Copy an operand into a contiguous temp with index order `order`.
  int64_t tmp_used = 0;
  const int64_t need = A0.numel() + B0.numel() + C0.numel();
  cplx* tmp_base = nullptr;
  auto take = [&](int64_t n) {
    if (!tmp_base) tmp_base = scratch(need);
    cplx* p = tmp_base + tmp_used;
    tmp_used += n;
    return p;
  };

  // Decide split points; relayout operands whose groups need more than one break.
  auto split_of = [&](const Operand& x, const Operand& y, const std::string& g, int& sp) -> int {
    // returns 0 ok, 1 x needs relayout, 2 y needs relayout
    std::vector<int> bx = breaks(x, g, ext), by = breaks(y, g, ext);
    std::vector<int> u = bx;
    for (int b : by)
      if (std::find(u.begin(), u.end(), b) == u.end()) u.push_back(b);
    if (u.size() <= 1) {
      sp = u.empty() ? 0 : u[0];
      return 0;
    }
    return bx.size() >= by.size() ? 1 : 2;
  };

  bool copyA = false, copyB = false, copyC = false;
  // batch group must be a single run in every operand
  if (!breaks(oa, gb, ext).empty()) copyA = true;
  if (!breaks(ob, gb, ext).empty()) copyB = true;
  if (!breaks(oc, gb, ext).empty()) copyC = true;
  int spm = 0, spn = 0, spk = 0;
  for (int round = 0; round < 4; ++round) {
    int r;
    bool changed = false;
    if ((r = split_of(oa, oc, gm, spm)) != 0) {
      if (r == 1 && !copyA) copyA = changed = true;
      else if (r == 2 && !copyC) copyC = changed = true;
      else if (!copyA) copyA = changed = true;
      else if (!copyC) copyC = changed = true;
    }
    if ((r = split_of(ob, oc, gn, spn)) != 0) {
      if (r == 1 && !copyB) copyB = changed = true;
      else if (r == 2 && !copyC) copyC = changed = true;
      else if (!copyB) copyB = changed = true;
      else if (!copyC) copyC = changed = true;
    }
    if ((r = split_of(oa, ob, gk, spk)) != 0) {
      if (r == 1 && !copyA) copyA = changed = true;
      else if (r == 2 && !copyB) copyB = changed = true;
      else if (!copyA) copyA = changed = true;
      else if (!copyB) copyB = changed = true;
    }
    if (copyA && oa.idx != gb + gm + gk) {
      View t = raw(take(A.numel()), [&] {
        std::vector<int64_t> s;
        for (char c : gb + gm + gk) s.push_back(ext.at(c));
        return s;
      }());
      std::vector<int> perm;
      for (char c : gb + gm + gk) perm.push_back((int)oa.idx.find(c));
      fill(t.p, t.numel(), cplx{0, 0}, stream);
      View src = permute(A, perm);
      AxpyDesc d;
      d.nd = t.nd;
      for (int k = 0; k < t.nd; ++k) {
        d.shape[k] = t.sh[k];
        d.sx[k] = src.st[k];
        d.sy[k] = t.st[k];
      }
      d.X = src.p;
      d.Y = t.p;
      d.alpha = cplx{1, 0};
      axpy_strided(d, stream);
      A = t;
      oa.idx = gb + gm + gk;
      changed = true;
    }
    if (copyB && ob.idx != gb + gk + gn) {
      View t = raw(take(B.numel()), [&] {
        std::vector<int64_t> s;
        for (char c : gb + gk + gn) s.push_back(ext.at(c));
        return s;
      }());
      std::vector<int> perm;
      for (char c : gb + gk + gn) perm.push_back((int)ob.idx.find(c));
      fill(t.p, t.numel(), cplx{0, 0}, stream);
      View src = permute(B, perm);
      AxpyDesc d;
      d.nd = t.nd;
      for (int k = 0; k < t.nd; ++k) {
        d.shape[k] = t.sh[k];
        d.sx[k] = src.st[k];
        d.sy[k] = t.st[k];
      }
      d.X = src.p;
      d.Y = t.p;
      d.alpha = cplx{1, 0};
      axpy_strided(d, stream);
      B = t;
      ob.idx = gb + gk + gn;
      changed = true;
    }
    if (!changed) break;
  }
  View Cfinal = C0;
  if (copyC) {
    std::vector<int64_t> s;
    for (char c : gb + gm + gn) s.push_back(ext.at(c));
    C = raw(take(extent(gb + gm + gn, ext)), s);
    fill(C.p, C.numel(), cplx{0, 0}, stream);
    oc.idx = gb + gm + gn;
  }
  // final split points (all operands now compatible)
  RTCC3_CHECK(split_of(oa, oc, gm, spm) == 0 && split_of(ob, oc, gn, spn) == 0 && split_of(oa, ob, gk, spk) == 0,
              "einsum: could not map " + spec);

  GemmDesc g;
  std::memset(&g, 0, sizeof(g));
  g.M = (int)extent(gm, ext);
  g.N = (int)extent(gn, ext);
  g.K = (int)extent(gk, ext);
  g.batch = (int)extent(gb, ext);
  int64_t t1, t0;
  int64_t m0a, n0b, k0a, m0c, n0c, k0b;
  level_strides(oa, gm, spm, ext, m0a, g.sAm1, g.sAm0);
  level_strides(oc, gm, spm, ext, m0c, g.sCm1, g.sCm0);
  level_strides(ob, gn, spn, ext, n0b, g.sBn1, g.sBn0);
  level_strides(oc, gn, spn, ext, n0c, g.sCn1, g.sCn0);
  level_strides(oa, gk, spk, ext, k0a, g.sAk1, g.sAk0);
  level_strides(ob, gk, spk, ext, k0b, g.sBk1, g.sBk0);
  g.M0 = (int)m0a;
  g.N0 = (int)n0b;
  g.K0 = (int)k0a;
  level_strides(oa, gb, 0, ext, t0, t1, g.sAb);
  level_strides(ob, gb, 0, ext, t0, t1, g.sBb);
  level_strides(oc, gb, 0, ext, t0, t1, g.sCb);
  g.A = A.p;
  g.B = B.p;
  g.C = C.p;
  g.alpha = alpha;
  g.prec = prec;
  if (g.K == 0) return;
  // host-side guard: the GEMM must not reach beyond the extent of its views
  auto reach = [](int64_t X, int64_t X0, int64_t s1, int64_t s0) -> int64_t {
    if (X <= 0) return 0;
    RTCC3_CHECK(X0 >= 1 && X % X0 == 0 && s1 >= 0 && s0 >= 0, "einsum: bad decomposition");
    return (X / X0 - 1) * s1 + (X0 - 1) * s0;
  };
  auto extent_of = [](const View& x) {
    int64_t m = 0;
    for (int k = 0; k < x.nd; ++k) {
      RTCC3_CHECK(x.st[k] >= 0, "einsum: negative stride");
      m += (x.sh[k] - 1) * x.st[k];
    }
    return m;
  };
  RTCC3_CHECK(reach(g.M, g.M0, g.sAm1, g.sAm0) + reach(g.K, g.K0, g.sAk1, g.sAk0) +
                      (int64_t)(g.batch - 1) * g.sAb <= extent_of(A),
              "einsum: A access out of range in " + spec);
  RTCC3_CHECK(reach(g.K, g.K0, g.sBk1, g.sBk0) + reach(g.N, g.N0, g.sBn1, g.sBn0) +
                      (int64_t)(g.batch - 1) * g.sBb <= extent_of(B),
              "einsum: B access out of range in " + spec);
  RTCC3_CHECK(reach(g.M, g.M0, g.sCm1, g.sCm0) + reach(g.N, g.N0, g.sCn1, g.sCn0) +
                      (int64_t)(g.batch - 1) * g.sCb <= extent_of(C),
              "einsum: C access out of range in " + spec);
  gemm(g, stream);
  if (copyC) {
    // scatter the temp result into the real output
    std::vector<int> perm;
    for (char c : sc) perm.push_back((int)oc.idx.find(c));
    View src = permute(C, perm);
    AxpyDesc d;
    d.nd = Cfinal.nd;
    for (int k = 0; k < Cfinal.nd; ++k) {
      d.shape[k] = Cfinal.sh[k];
      d.sx[k] = src.st[k];
      d.sy[k] = Cfinal.st[k];
    }
    d.X = src.p;
    d.Y = Cfinal.p;
    d.alpha = cplx{1, 0};
    axpy_strided(d, stream);
  }
}

}  // namespace rtcc3
