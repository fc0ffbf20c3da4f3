// Instantiates the FFT kernels of fft_kernels.h for one size, PMR_FFT_SIZE (one
// translation unit per size keeps the build parallel).
#include "fft_kernels.h"

#ifndef PMR_FFT_SIZE
#error "compile with -DPMR_FFT_SIZE=<n>"
#endif
#define PMR_CAT2(a, b) a##b
#define PMR_CAT(a, b) PMR_CAT2(a, b)

namespace pmr {

void PMR_CAT(fft_zr2c_, PMR_FFT_SIZE)(int fields, const float* in, FieldMap im, const float* in2,
                                      float a1, float a2, const double* sc, float2* out,
                                      FieldMap om, hipStream_t s) {
  zr2c<PMR_FFT_SIZE>(fields, in, im, in2, a1, a2, sc, out, om, s);
}

void PMR_CAT(fft_zc2r_, PMR_FFT_SIZE)(int fields, const float2* in, FieldMap im, float* out,
                                      FieldMap om, const float* add, hipStream_t s) {
  zc2r<PMR_FFT_SIZE>(fields, in, im, out, om, add, s);
}

void PMR_CAT(fft_zc2r3_, PMR_FFT_SIZE)(int items, const float2* in, FieldMap im, Vec3* out,
                                       size_t out_item_stride, hipStream_t s) {
  zc2r3<PMR_FFT_SIZE>(items, in, im, out, out_item_stride, s);
}

void PMR_CAT(fft_paint_r2c_, PMR_FFT_SIZE)(int channels, const PaintArgs& a, int batch,
                                           float2* out, FieldMap om, hipStream_t s) {
  if (channels == 3)
    paint_r2c<3, PMR_FFT_SIZE>(a, batch, out, om, s);
  else
    paint_r2c<1, PMR_FFT_SIZE>(a, batch, out, om, s);
}

void PMR_CAT(fft_ypass_, PMR_FFT_SIZE)(int fields, float2* d, FieldMap m, bool inv,
                                       hipStream_t s, KzWin win) {
  ypass<PMR_FFT_SIZE>(fields, d, m, inv, s, win);
}

void PMR_CAT(fft_xpass_, PMR_FFT_SIZE)(int op, const XPassArgs& a, hipStream_t s) {
  xpass_dispatch<PMR_FFT_SIZE>(op, a, s);
}

}  // namespace pmr
