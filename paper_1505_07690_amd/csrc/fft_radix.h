// In-register small DFTs for the Stockham passes (radix 2, 3, 4, 5, 8, 16).
// sgn = -1 gives the forward kernel exp(-2 pi i jk / R), +1 the inverse.
#pragma once
#include <hip/hip_runtime.h>

namespace os3d {

__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ float2 cscale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }
__device__ __forceinline__ float2 cconj(float2 a) { return make_float2(a.x, -a.y); }
// multiply by sgn * i
__device__ __forceinline__ float2 cmul_si(float2 a, float sgn) { return make_float2(-sgn * a.y, sgn * a.x); }

__device__ __forceinline__ void dft2(float2* v) {
  float2 a = v[0], b = v[1];
  v[0] = cadd(a, b);
  v[1] = csub(a, b);
}

__device__ __forceinline__ void dft4(float2& x0, float2& x1, float2& x2, float2& x3, float sgn) {
  float2 t0 = cadd(x0, x2), t1 = csub(x0, x2), t2 = cadd(x1, x3), t3 = cmul_si(csub(x1, x3), sgn);
  x0 = cadd(t0, t2);
  x2 = csub(t0, t2);
  x1 = cadd(t1, t3);
  x3 = csub(t1, t3);
}

__device__ __forceinline__ void dft3(float2* v, float sgn) {
  const float s3 = 0.866025403784438646764f * sgn;
  float2 t1 = cadd(v[1], v[2]), t2 = csub(v[1], v[2]);
  float2 m = make_float2(v[0].x - 0.5f * t1.x, v[0].y - 0.5f * t1.y);
  float2 it = make_float2(-s3 * t2.y, s3 * t2.x);
  v[0] = cadd(v[0], t1);
  v[1] = cadd(m, it);
  v[2] = csub(m, it);
}

__device__ __forceinline__ void dft5(float2* v, float sgn) {
  const float c1 = 0.309016994374947424102f, c2 = -0.809016994374947424102f;
  const float s1 = 0.951056516295153572116f * sgn, s2 = 0.587785252292473129169f * sgn;
  float2 t1 = cadd(v[1], v[4]), t2 = cadd(v[2], v[3]), t3 = csub(v[1], v[4]), t4 = csub(v[2], v[3]);
  float2 a1 = make_float2(v[0].x + c1 * t1.x + c2 * t2.x, v[0].y + c1 * t1.y + c2 * t2.y);
  float2 a2 = make_float2(v[0].x + c2 * t1.x + c1 * t2.x, v[0].y + c2 * t1.y + c1 * t2.y);
  float2 b1 = make_float2(s1 * t3.x + s2 * t4.x, s1 * t3.y + s2 * t4.y);
  float2 b2 = make_float2(s2 * t3.x - s1 * t4.x, s2 * t3.y - s1 * t4.y);
  v[0] = cadd(v[0], cadd(t1, t2));
  // i * b = (-b.y, b.x)
  v[1] = make_float2(a1.x - b1.y, a1.y + b1.x);
  v[4] = make_float2(a1.x + b1.y, a1.y - b1.x);
  v[2] = make_float2(a2.x - b2.y, a2.y + b2.x);
  v[3] = make_float2(a2.x + b2.y, a2.y - b2.x);
}

__device__ __forceinline__ void dft8(float2* v, float sgn) {
  const float r = 0.707106781186547524401f;
  float2 e0 = v[0], e1 = v[2], e2 = v[4], e3 = v[6];
  float2 o0 = v[1], o1 = v[3], o2 = v[5], o3 = v[7];
  dft4(e0, e1, e2, e3, sgn);
  dft4(o0, o1, o2, o3, sgn);
  // W8^k = exp(sgn i pi k / 4)
  float2 w1o = make_float2(r * (o1.x - sgn * o1.y), r * (o1.y + sgn * o1.x));
  float2 w2o = cmul_si(o2, sgn);
  float2 w3o = make_float2(r * (-o3.x - sgn * o3.y), r * (-o3.y + sgn * o3.x));
  v[0] = cadd(e0, o0);
  v[4] = csub(e0, o0);
  v[1] = cadd(e1, w1o);
  v[5] = csub(e1, w1o);
  v[2] = cadd(e2, w2o);
  v[6] = csub(e2, w2o);
  v[3] = cadd(e3, w3o);
  v[7] = csub(e3, w3o);
}

// 16 = 4 x 4: inner DFT4 over n1 (stride 4), twiddle W16^(n2 k1), outer DFT4 over n2.
__device__ __forceinline__ void dft16(float2* v, float sgn) {
  const float c1 = 0.923879532511286756128f, s1 = 0.382683432365089771728f, r = 0.707106781186547524401f;
#pragma unroll
  for (int n2 = 0; n2 < 4; ++n2) dft4(v[n2], v[4 + n2], v[8 + n2], v[12 + n2], sgn);
  // now v[4*k1 + n2] = A[n2][k1]; multiply by W16^(n2 k1) = exp(sgn i 2 pi n2 k1 / 16)
  const float2 w[10] = {make_float2(1.f, 0.f),  make_float2(c1, sgn * s1), make_float2(r, sgn * r),
                        make_float2(s1, sgn * c1), make_float2(0.f, sgn),    make_float2(-s1, sgn * c1),
                        make_float2(-r, sgn * r), make_float2(-c1, sgn * s1), make_float2(-1.f, 0.f),
                        make_float2(-c1, -sgn * s1)};
#pragma unroll
  for (int k1 = 1; k1 < 4; ++k1)
#pragma unroll
    for (int n2 = 1; n2 < 4; ++n2) v[4 * k1 + n2] = cmul(v[4 * k1 + n2], w[n2 * k1]);
  float2 o[16];
#pragma unroll
  for (int k1 = 0; k1 < 4; ++k1) {
    float2 a0 = v[4 * k1], a1 = v[4 * k1 + 1], a2 = v[4 * k1 + 2], a3 = v[4 * k1 + 3];
    dft4(a0, a1, a2, a3, sgn);
    o[k1] = a0;
    o[k1 + 4] = a1;
    o[k1 + 8] = a2;
    o[k1 + 12] = a3;
  }
#pragma unroll
  for (int i = 0; i < 16; ++i) v[i] = o[i];
}

template <int R>
__device__ __forceinline__ void dft_r(float2* v, float sgn) {
  if constexpr (R == 2) {
    dft2(v);
  } else if constexpr (R == 3) {
    dft3(v, sgn);
  } else if constexpr (R == 4) {
    dft4(v[0], v[1], v[2], v[3], sgn);
  } else if constexpr (R == 5) {
    dft5(v, sgn);
  } else if constexpr (R == 8) {
    dft8(v, sgn);
  } else if constexpr (R == 16) {
    dft16(v, sgn);
  }
}

}  // namespace os3d
