// Slab-solver internals: device vector kernels and layout conversions.
#pragma once

#include "internal.h"

namespace stdg {

constexpr int kMaxBasis = 32;   // restart + 1 <= 32
constexpr int kDotBlocks = 1024;

int blas_multi_dot(const double* V, int64_t ld, int k, const void* w, bool w_f32, int64_t n, double* partial,
                   double* out, hipStream_t s);
int blas_update(double* w, const void* src, bool src_f32, const double* V, int64_t ld, int k, const double* h,
                int64_t n, hipStream_t s);
int blas_scale(double* out, const double* in, double alpha, int64_t n, hipStream_t s);
int blas_lincomb(void* out, bool out_f32, const double* V, int64_t ld, int k, const double* y, int64_t n,
                 hipStream_t s);
int blas_axpy(double* y, const double* x, double a, int64_t n, hipStream_t s);
int blas_to_f32(float* out, const double* in, double alpha, int64_t n, hipStream_t s);
int layout_embed(const Mesh* m, double* U, const double* x, const double* st, hipStream_t s);
int layout_level(const Mesh* m, double* st, const double* x, int lev, hipStream_t s);
int layout_guess(const Mesh* m, double* x, const double* st, hipStream_t s);
int energy_async(const Mesh* m, const double* state, double* d_partial, double* d_out, hipStream_t s);
int ensure_state_off(Mesh* m);

}  // namespace stdg
