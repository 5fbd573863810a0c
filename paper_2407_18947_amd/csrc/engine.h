// Tensor views, an einsum-style contraction engine on the batched MFMA GEMM,
// and a reverse-mode tape over its operations.
#pragma once

#include <map>
#include <string>
#include <vector>

#include "common.h"

namespace rtcc3 {

// A strided view into a device buffer owned by the Engine.
struct View {
  cplx* p = nullptr;
  int nd = 0;
  int64_t sh[8] = {0};
  int64_t st[8] = {0};
  int buf = -1;     // owning buffer id (-1: untracked memory)
  int64_t off = 0;  // element offset of p inside the buffer
  int64_t numel() const {
    int64_t n = 1;
    for (int k = 0; k < nd; ++k) n *= sh[k];
    return n;
  }
};

class Engine {
 public:
  explicit Engine(hipStream_t s) : stream(s) {}
  ~Engine();
  Engine(const Engine&) = delete;
  Engine& operator=(const Engine&) = delete;

  hipStream_t stream;
  int prec = 0;  // GEMM precision used by einsum (0 = FP64)

  // Once sealed, a request that would allocate device memory (a new named
  // buffer, a larger scratch, a first gradient) throws ESTATE instead: the
  // context allocates everything it needs at creation, so nothing is
  // allocated while amplitudes are propagated.
  void seal(bool on) { sealed_ = on; }

  // Named buffers, allocated once and reused (get-or-create).
  int buffer(const std::string& name, int64_t n);
  // Free a named buffer after the stream has drained (the name may then be
  // requested again with another size); views into it become invalid.
  void release(const std::string& name);
  View tensor(const std::string& name, std::vector<int64_t> shape);  // contiguous, zeroed on request
  View tensor_of(int buf, std::vector<int64_t> shape);
  void zero(const View& v);
  void zero_buffer(int buf);
  cplx* data(int buf) { return bufs_[buf].p; }
  int64_t size(int buf) { return bufs_[buf].n; }

  static View slice(View v, int dim, int64_t lo, int64_t hi);
  static View permute(View v, std::vector<int> perm);  // out dim d = in dim perm[d]
  static View diag(View v, int d0, int d1);             // diagonal of dims d0,d1 (equal extents) at d0
  static View raw(cplx* p, std::vector<int64_t> shape); // untracked contiguous view

  // C += alpha * einsum(spec, A, B).  Every index of A (B) must appear in B (A)
  // or in C; spec like "ijcd,acbd->ijab".
  void einsum(const char* spec, cplx alpha, const View& A, const View& B, const View& C);
  // Y += alpha * X elementwise (same shape; either may be a permuted view).
  void axpy(cplx alpha, const View& X, const View& Y);

  // Reverse mode.  Buffers flagged with requires_grad propagate the flag to
  // the outputs of recorded operations; backward() then accumulates
  // gradients (holomorphic derivatives) into shadow buffers.
  void set_requires_grad(int buf, bool on);
  bool requires_grad(int buf) const { return buf >= 0 && bufs_[buf].rg; }
  View grad(const View& v);
  void tape_begin();
  void tape_end() { recording_ = false; }
  void tape_resume() { recording_ = true; }  // continue the current tape (after a pause with tape_end)
  void zero_grads();
  void backward();

  // Tangent (forward) mode.  Once twins are enabled every buffer and every
  // gradient has a twin of its size, meant to hold its derivative along one
  // direction.  While tangent mode is on, each operation also applies its
  // derivative: einsum C += a A.B adds a (A'.B + A.B') to C', axpy Y += a X
  // adds a X' to Y', zero() clears the twin, copy() copies it, and the reverse
  // sweep differentiates its own operations the same way, so the twins of the
  // gradients become the derivatives of the gradients.  A twin is looked up
  // by address (any pointer into a buffer or gradient).  A twin never written
  // since it was last cleared is known to be zero (constants) and skipped.
  void enable_twins();
  bool twins() const { return twins_; }
  void set_tangent(bool on) { tangent_ = on && twins_; }
  bool tangent() const { return tangent_; }
  // Twin of the element at p for reading: nullptr when it is zero (or p lies
  // outside every buffer).
  const cplx* twin(const cplx* p) const;
  // Twin of the element at p for writing (from then on it is not known to be
  // zero); p must lie in a buffer or gradient.
  cplx* twin_out(const cplx* p);
  // dst[0..n) = src[0..n), with the twins when tangent mode is on (a zero twin
  // of src clears that of dst).
  void copy(cplx* dst, const cplx* src, int64_t n);

 private:
  struct Buf {
    std::string name;
    cplx* p = nullptr;
    cplx* g = nullptr;
    int64_t n = 0;
    bool rg = false;
    cplx* tp = nullptr;  // twin of p
    cplx* tg = nullptr;  // twin of g
    bool tp_nz = false, tg_nz = false;  // twin written since it was last cleared
  };
  // address range of a buffer (kind 0) or gradient (kind 1)
  struct Range {
    int64_t n;
    int buf;
    int kind;
  };
  std::map<const cplx*, Range> ranges_;
  bool twins_ = false, tangent_ = false;
  const Range* find(const cplx* p, int64_t* off) const;
  cplx* alloc_twin(int64_t n);
  void einsum_dual(const std::string& spec, cplx alpha, const View& A, const View& B, const View& C);
  void axpy_exec(cplx alpha, const View& X, const View& Y);
  struct Op {
    int kind;  // 0 einsum, 1 axpy
    std::string spec;
    cplx alpha;
    View A, B, C;
  };
  std::vector<Buf> bufs_;
  std::map<std::string, int> names_;
  std::vector<Op> tape_;
  bool recording_ = false;
  bool sealed_ = false;
  // Relayout scratch, one region per stream that einsums run on, so that
  // einsums on different streams may run at the same time.
  struct Scratch {
    hipStream_t stream;
    cplx* p;
    int64_t n;
  };
  std::vector<Scratch> scratch_;

  cplx* scratch(int64_t n);
  void einsum_exec(const std::string& spec, cplx alpha, const View& A, const View& B, const View& C);
};

}  // namespace rtcc3
