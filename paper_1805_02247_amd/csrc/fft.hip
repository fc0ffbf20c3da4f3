// Host dispatch of the 3-D FFT passes over the supported sizes, and the tile-shape table.
// The kernels live in fft_kernels.h, instantiated per size by fft_size.hip.
#include "pmr_internal.h"

namespace pmr {

TileShape g_fft_tile[3][10] = {
    {{16, 256, 0}, {16, 256, 0}, {16, 256, 0}, {16, 256, 0}, {16, 256, 0}, {16, 256, 0},
     {16, 256, 0}, {16, 256, 0}, {16, 256, 0}, {16, 256, 0}},
    {{16, 256, 0}, {16, 256, 0}, {16, 256, 0}, {16, 256, 0}, {16, 256, 0}, {16, 256, 0},
     {16, 256, 0}, {16, 256, 0}, {16, 256, 0}, {16, 256, 0}},
    {{16, 256, 0}, {16, 256, 0}, {16, 256, 0}, {16, 256, 0}, {16, 256, 0}, {16, 256, 0},
     {16, 256, 0}, {16, 256, 0}, {16, 256, 0}, {16, 256, 0}}};

namespace {
int log2i(int n) {
  int l = 0;
  while ((1 << l) < n) ++l;
  return l;
}
}  // namespace

void fft_zr2c_16(int, const float*, FieldMap, const float*, float, float, const double*, float2*,
               FieldMap, hipStream_t);
void fft_zc2r_16(int, const float2*, FieldMap, float*, FieldMap, const float*, hipStream_t);
void fft_zc2r3_16(int, const float2*, FieldMap, Vec3*, size_t, hipStream_t);
void fft_paint_r2c_16(int, const PaintArgs&, int, float2*, FieldMap, hipStream_t);
void fft_ypass_16(int, float2*, FieldMap, bool, hipStream_t, KzWin);
void fft_xpass_16(int, const XPassArgs&, hipStream_t);
void fft_zr2c_32(int, const float*, FieldMap, const float*, float, float, const double*, float2*,
               FieldMap, hipStream_t);
void fft_zc2r_32(int, const float2*, FieldMap, float*, FieldMap, const float*, hipStream_t);
void fft_zc2r3_32(int, const float2*, FieldMap, Vec3*, size_t, hipStream_t);
void fft_paint_r2c_32(int, const PaintArgs&, int, float2*, FieldMap, hipStream_t);
void fft_ypass_32(int, float2*, FieldMap, bool, hipStream_t, KzWin);
void fft_xpass_32(int, const XPassArgs&, hipStream_t);
void fft_zr2c_64(int, const float*, FieldMap, const float*, float, float, const double*, float2*,
               FieldMap, hipStream_t);
void fft_zc2r_64(int, const float2*, FieldMap, float*, FieldMap, const float*, hipStream_t);
void fft_zc2r3_64(int, const float2*, FieldMap, Vec3*, size_t, hipStream_t);
void fft_paint_r2c_64(int, const PaintArgs&, int, float2*, FieldMap, hipStream_t);
void fft_ypass_64(int, float2*, FieldMap, bool, hipStream_t, KzWin);
void fft_xpass_64(int, const XPassArgs&, hipStream_t);
void fft_zr2c_128(int, const float*, FieldMap, const float*, float, float, const double*, float2*,
               FieldMap, hipStream_t);
void fft_zc2r_128(int, const float2*, FieldMap, float*, FieldMap, const float*, hipStream_t);
void fft_zc2r3_128(int, const float2*, FieldMap, Vec3*, size_t, hipStream_t);
void fft_paint_r2c_128(int, const PaintArgs&, int, float2*, FieldMap, hipStream_t);
void fft_ypass_128(int, float2*, FieldMap, bool, hipStream_t, KzWin);
void fft_xpass_128(int, const XPassArgs&, hipStream_t);
void fft_zr2c_256(int, const float*, FieldMap, const float*, float, float, const double*, float2*,
               FieldMap, hipStream_t);
void fft_zc2r_256(int, const float2*, FieldMap, float*, FieldMap, const float*, hipStream_t);
void fft_zc2r3_256(int, const float2*, FieldMap, Vec3*, size_t, hipStream_t);
void fft_paint_r2c_256(int, const PaintArgs&, int, float2*, FieldMap, hipStream_t);
void fft_ypass_256(int, float2*, FieldMap, bool, hipStream_t, KzWin);
void fft_xpass_256(int, const XPassArgs&, hipStream_t);
void fft_zr2c_512(int, const float*, FieldMap, const float*, float, float, const double*, float2*,
               FieldMap, hipStream_t);
void fft_zc2r_512(int, const float2*, FieldMap, float*, FieldMap, const float*, hipStream_t);
void fft_zc2r3_512(int, const float2*, FieldMap, Vec3*, size_t, hipStream_t);
void fft_paint_r2c_512(int, const PaintArgs&, int, float2*, FieldMap, hipStream_t);
void fft_ypass_512(int, float2*, FieldMap, bool, hipStream_t, KzWin);
void fft_xpass_512(int, const XPassArgs&, hipStream_t);

#define PMR_FOR_N(MACRO) \
  MACRO(16) MACRO(32) MACRO(64) MACRO(128) MACRO(256) MACRO(512)

void launch_zpass_r2c(int n, int fields, const float* in, FieldMap im, const float* in2, float a1,
                      float a2, const double* scale_dev, float2* out, FieldMap om, hipStream_t s) {
  switch (n) {
#define CASE(NN) \
  case NN: fft_zr2c_##NN(fields, in, im, in2, a1, a2, scale_dev, out, om, s); break;
    PMR_FOR_N(CASE)
#undef CASE
    default: break;
  }
}

void launch_zpass_c2r(int n, int fields, const float2* in, FieldMap im, float* out, FieldMap om,
                      const float* add, hipStream_t s) {
  switch (n) {
#define CASE(NN) \
  case NN: fft_zc2r_##NN(fields, in, im, out, om, add, s); break;
    PMR_FOR_N(CASE)
#undef CASE
    default: break;
  }
}

void launch_zpass_c2r3(int n, int items, const float2* in, FieldMap im, Vec3* out,
                       size_t out_item_stride, hipStream_t s) {
  switch (n) {
#define CASE(NN) \
  case NN: fft_zc2r3_##NN(items, in, im, out, out_item_stride, s); break;
    PMR_FOR_N(CASE)
#undef CASE
    default: break;
  }
}

void launch_paint_r2c(int n, int channels, const PaintArgs& a, int batch, float2* out, FieldMap om,
                      hipStream_t s) {
  switch (n) {
#define CASE(NN) \
  case NN: fft_paint_r2c_##NN(channels, a, batch, out, om, s); break;
    PMR_FOR_N(CASE)
#undef CASE
    default: break;
  }
}

void launch_ypass(int n, int fields, float2* data, FieldMap m, bool inverse, hipStream_t s,
                  KzWin win) {
  switch (n) {
#define CASE(NN) \
  case NN: fft_ypass_##NN(fields, data, m, inverse, s, win); break;
    PMR_FOR_N(CASE)
#undef CASE
    default: break;
  }
}

int set_fft_tile(int n, int pass, int pc, int nth, int staging) {
  if (pass < 0 || pass > 2) return -1;
  if (n < 16 || n > 512 || (n & (n - 1))) return -1;
  if (pc != 8 && pc != 16 && pc != 32) return -1;
  if (nth != 256 && nth != 512) return -1;
  if (n * pc < nth || (n * pc + n) * 8 > 160 * 1024 || n * pc / nth > 16) return -1;
  if (staging < 0 || staging > 2) return -1;
  g_fft_tile[pass][log2i(n)] = {pc, nth, staging};
  return 0;
}

int g_fft_slab[10] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
int g_paint_rows[2][10] = {{0, 0, 0, 0, 0, 0, 0, 0, 0, 0}, {0, 0, 0, 0, 0, 0, 0, 0, 0, 0}};

int set_paint_rows(int n, int channels, int rows) {
  if (n < 16 || n > 512 || (n & (n - 1))) return -1;
  if (channels != 1 && channels != 3) return -1;
  if (rows != 0 && rows != 1 && rows != 2 && rows != 4 && rows != 8 && rows != 16) return -1;
  g_paint_rows[channels == 3][log2i(n)] = rows;
  return 0;
}

int get_paint_rows(int n, int channels) { return g_paint_rows[channels == 3][log2i(n)]; }

int set_fft_slab(int n, int columns) {
  if (n < 16 || n > 512 || (n & (n - 1))) return -1;
  if (columns < 0 || columns > 512 || (columns & (columns - 1))) return -1;
  g_fft_slab[log2i(n)] = columns;
  return 0;
}

int get_fft_slab(int n) { return g_fft_slab[log2i(n)]; }

// Columns of the kz window in which the y and x passes of one transform run back to back
// (0: each pass over the whole half spectrum): the requested width rounded up to a multiple
// of the column count of every strided pass at this size (all are powers of two), so that
// no chunk straddles two windows.
int fft_slab_columns(int n) {
  const int want = g_fft_slab[log2i(n)];
  if (want <= 0) return 0;
  int w = want;
  for (int pass = 0; pass < 3; ++pass) {
    const TileShape t = g_fft_tile[pass][log2i(n)];
    const bool ok = t.pc >= 8 && t.pc <= 32 && n * t.pc >= t.nth &&
                    (n * t.pc + n) * 8 <= 160 * 1024 && n * t.pc / t.nth <= 16;
    const int pc = ok ? t.pc : 16;  // the dispatch falls back to 16 columns
    if (pc > w) w = pc;
  }
  return w >= n / 2 + 1 ? 0 : w;
}

void get_fft_tile(int n, int pass, int* pc, int* nth, int* staging) {
  const TileShape t = g_fft_tile[pass][log2i(n)];
  *pc = t.pc;
  *nth = t.nth;
  *staging = t.staging;
}

void launch_xpass(int op, const XPassArgs& a, hipStream_t s) {
  switch (a.n) {
#define CASE(NN) \
  case NN: fft_xpass_##NN(op, a, s); break;
    PMR_FOR_N(CASE)
#undef CASE
    default: break;
  }
}

}  // namespace pmr
