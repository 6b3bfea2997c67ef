// Internal declarations of the PEIFE-linear library (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <string>
#include <vector>

#include "peifem.h"

namespace pe {

// Interior sizes are padded to a multiple of PAD in every device field so
// that the transform tiles never straddle a ragged edge; padding entries are
// kept at zero (the padded DST matrix has zero rows/columns there).
constexpr int PAD = 32;

inline int pad_up(int n) { return (n + PAD - 1) / PAD * PAD; }

struct Axis {
  int n = 0, np = 0;
  double lo = 0, hi = 0, h = 0;
  double *d_lam = nullptr;       // [n]   generalized eigenvalues lambda_a(k)
  double *d_sig = nullptr;       // [n]   1/sqrt(mu_a(k)), mu_a the mass eigenvalues
  double *d_S = nullptr;         // [np][np] orthonormal DST-I, zero padded
  uint16_t *d_Shi = nullptr;     // [np][np] bf16 high part of S
  uint16_t *d_Slo = nullptr;     // [np][np] bf16 low part of S (S - hi)
};

struct PendingTiming {
  hipEvent_t start, stop;
  int cls;
  double flops, bytes;
};

struct DevTerm {                 // a forcing term as the kernels read it
  double amp;
  double alpha, omega, phase;
  double p[4];
};

}  // namespace pe

struct pe_grid_s {
  int dim = 0;
  int precision = PE_FP64;
  int quad_q = 3;
  double D = 0;
  int64_t dof = 0;               // prod n_a
  int64_t dofp = 0;              // prod np_a (padded field size)
  pe::Axis ax[PE_MAX_DIM];
  int n_terms = 0;
  pe::DevTerm h_terms[PE_MAX_TERMS];
  pe::DevTerm *d_terms = nullptr;        // [n_terms]
  double *d_C[PE_MAX_DIM] = {nullptr, nullptr, nullptr};  // [n_terms][np_a] 1D loads
  // kernel timing (benchmark instrumentation)
  bool timing = false;
  std::vector<pe::PendingTiming> pending;
  pe_kernel_stat stats[PE_K_COUNT] = {};
};

namespace pe {

// ---------------------------------------------------------------- errors
pe_status set_error(pe_status st, const char *fmt, ...);
void clear_error();

#define PE_HIP(call)                                                              \
  do {                                                                            \
    hipError_t _e = (call);                                                       \
    if (_e != hipSuccess)                                                         \
      return ::pe::set_error(PE_E_HIP, "%s failed: %s (%s:%d)", #call,            \
                             hipGetErrorString(_e), __FILE__, __LINE__);          \
  } while (0)

#define PE_TRY(expr)                    \
  do {                                  \
    pe_status _s = (expr);              \
    if (_s != PE_OK) return _s;         \
  } while (0)

inline hipStream_t as_stream(void *s) { return reinterpret_cast<hipStream_t>(s); }

// ------------------------------------------------------------- workspace
// A bump allocator over the caller's workspace (256-byte aligned slices).
struct Arena {
  char *base;
  size_t size, off = 0;
  Arena(void *b, size_t s) : base(static_cast<char *>(b)), size(s) {}
  template <class T>
  T *take(size_t count) {
    size_t o = (off + 255) & ~size_t(255);
    size_t bytes = count * sizeof(T);
    if (o + bytes > size) return nullptr;
    off = o + bytes;
    return reinterpret_cast<T *>(base + o);
  }
  static size_t need(size_t bytes) { return (bytes + 255) & ~size_t(255); }
};

// ---------------------------------------------------------- field passes
// Per-field time stamps of a batch of stage fields: field f is slice
// n = n0 + f / (jc * s), step j = j0 + (f / s) % jc, stage i = f % s at time
// ((t0 + n*dT) + j*dt) + c_i*dt.
struct FieldBatch {
  int n0, nslices;      // slices in this batch
  int j0, jc;           // steps in this batch
  int s;                // stages
  double t0, dT, dt;
  double c[PE_MAX_STAGES];
  int64_t count() const { return int64_t(nslices) * jc * s; }
};

// Evaluate the load vectors of a batch of fields and transform them to DST
// coefficients (before the 1/sqrt(mu) scaling).  work0/work1 each hold
// batch.count() padded fields of the grid's stage type; coef holds
// count * n_terms doubles.  Returns the buffer holding the result.
pe_status load_and_transform(pe_grid g, const FieldBatch &b, void *work0, void *work1,
                             double *coef, void **result, hipStream_t st);

// Per-axis DST products of `count` padded fields (FP64): in -> out, d passes
// ping-ponging between the two buffers; *result receives the final buffer.
pe_status dst_fields_f64(pe_grid g, int64_t count, double *buf0, double *buf1, double **result,
                         hipStream_t st);
pe_status dst_fields_split(pe_grid g, int64_t count, float *buf0, float *buf1, float **result,
                           hipStream_t st);

// bytes of one padded stage field
size_t field_bytes(pe_grid g);

// Brackets the launches made during its lifetime with HIP events when the
// grid's timing is enabled (no-op otherwise).
struct TimedScope {
  pe_grid g;
  hipStream_t st;
  PendingTiming pt{};
  bool on;
  TimedScope(pe_grid g_, int cls, double flops, double bytes, hipStream_t s)
      : g(g_), st(s), on(g_->timing) {
    if (!on) return;
    pt.cls = cls;
    pt.flops = flops;
    pt.bytes = bytes;
    if (hipEventCreate(&pt.start) != hipSuccess || hipEventCreate(&pt.stop) != hipSuccess ||
        hipEventRecord(pt.start, st) != hipSuccess)
      on = false;
  }
  ~TimedScope() {
    if (!on) return;
    if (hipEventRecord(pt.stop, st) == hipSuccess) g->pending.push_back(pt);
  }
};

}  // namespace pe
