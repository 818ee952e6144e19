// Internal interface between the C ABI layer (abi.hip) and the warm-start
// network's kernels (cnn.hip).  Tensors are [C][D][H][W] float32, W fastest.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pct {
namespace cnn {

hipError_t conv3d(const float *x, const float *w, const float *b, float *y, int cin, int cout, int D, int H, int W,
                  hipStream_t s);
hipError_t flip_weights(const float *w, float *wt, int cin, int cout, hipStream_t s);
// BF16 matrix-core convolution (cin % 8 == 0, cout % 16 == 0); wpack: scratch
// of mfma_pack_bytes(cin, cout) bytes for the packed weights
bool mfma_shape_ok(int cin, int cout);
int64_t mfma_pack_bytes(int cin, int cout);
hipError_t conv3d_mfma(const float *x, const float *w, const float *b, float *y, void *wpack, int cin, int cout,
                       int D, int H, int W, hipStream_t s);
int64_t wgrad_chunks(int D, int H, int W);
hipError_t conv3d_wgrad(const float *x, const float *dy, float *dw, float *db, float *part, int cin, int cout, int D,
                        int H, int W, hipStream_t s);
// BF16 matrix-core weight gradient (cin % 16 == 0, cout % 16 == 0): part
// holds wgrad_mfma_slabs(...) x cout x (cin * 27 + 1) floats
bool mfma_wgrad_ok(int cin, int cout);
int64_t wgrad_mfma_slabs(int cin, int cout, int D, int H, int W);
hipError_t conv3d_wgrad_mfma(const float *x, const float *dy, float *dw, float *db, float *part, int cin, int cout,
                             int D, int H, int W, hipStream_t s);
hipError_t relu(const float *x, float *y, int64_t n, hipStream_t s);
hipError_t relu_bwd(const float *y, const float *dy, float *dx, int64_t n, hipStream_t s);
hipError_t pool(const float *x, float *y, int C, int D, int H, int W, hipStream_t s);
hipError_t pool_bwd(const float *dy, float *dx, int C, int D, int H, int W, hipStream_t s);
hipError_t upsample(const float *x, float *y, int C, int d, int h, int w, hipStream_t s);
hipError_t upsample_bwd(const float *dy, float *dx, int C, int d, int h, int w, hipStream_t s);
hipError_t add(const float *a, const float *b, float *y, int64_t n, hipStream_t s);
hipError_t axpy(float a, const float *x, float *y, int64_t n, hipStream_t s);
hipError_t mask(const float *x, const uint8_t *m, float *y, int64_t n, hipStream_t s);
int64_t mse_parts(int64_t n);
hipError_t mse(const float *y, const float *t, float *dy, double *part, double *loss, int64_t n, hipStream_t s);
hipError_t adam(float *w, const float *g, float *m, float *v, int64_t n, float lr, float b1, float b2, float eps,
                int step, hipStream_t s);

}  // namespace cnn
}  // namespace pct
