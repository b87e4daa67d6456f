// A recorded sequence of kernel launches ("program") whose descriptors live
// in one device blob.  A sweep of the fit is recorded once per distinct
// shape plan and then replayed eagerly or as a captured hipGraph.
#pragma once

#include <cstring>
#include <map>
#include <string>
#include <vector>

#include "fitkern.hpp"
#include "gemm.hpp"
#include "linalg.hpp"

namespace mpofit {

enum class LK { Gemm, Chol, Trsm, Eig, Omega, Sign, Scale, Perm, Sval, Fill, Norm, Bump, Jacobi, NormBig, Geqr, Naive, Polish, Orgqr, Trunc, Hhqr };

struct Launch {
  LK kind;
  GemmKind gk{};
  size_t off = 0;       // byte offset of the descriptors in the blob
  int n = 0;            // descriptor count
  long long wgs = 0;    // GEMM workgroups
  long long maxa = 0;   // per-kind size hint (rows, elements, ...)
  int maxb = 0;
  int* counter = nullptr;  // Bump target
  void* aux = nullptr;     // NormBig: partial-sum buffer
  int bump_by = 0;
  std::string cls;      // kernel class for profiling
  double flops = 0;     // algorithmic flops credited to this launch
};

struct Program {
  std::vector<Launch> launches;
  std::vector<unsigned char> blob;
  char* dev = nullptr;  // device copy of blob (inside the workspace)
  size_t dev_cap = 0;

  template <class D>
  size_t push(const std::vector<D>& ds) {
    size_t off = (blob.size() + 63) & ~size_t(63);
    blob.resize(off + ds.size() * sizeof(D));
    std::memcpy(blob.data() + off, ds.data(), ds.size() * sizeof(D));
    return off;
  }
  template <class D>
  const D* host(const Launch& l) const {
    return reinterpret_cast<const D*>(blob.data() + l.off);
  }
  template <class D>
  const D* device(const Launch& l) const {
    return reinterpret_cast<const D*>(dev + l.off);
  }
};

// Enqueues every launch of `p` on `s`; when `ev` is non-null, records an
// event after each launch (ev must hold launches.size()+1 events).
void run_program(const Program& p, hipStream_t s, hipEvent_t* ev);

}  // namespace mpofit
