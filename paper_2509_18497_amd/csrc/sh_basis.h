// Real spherical harmonics up to degree 3 (K = 1, 4, 9, 16 coefficients)
// in the order Y00, Y1-1, Y10, Y11, Y2-2, ..., Y33 (Sec. 3.2), as the
// closed-form polynomials of a unit vector (x, y, z) in a surfel's tangent
// frame (t_u, t_v, n); Condon-Shortley phase folded in, so that
// Y1-1 ~ y, Y10 ~ z, Y11 ~ x.
#pragma once

#include <hip/hip_runtime.h>

namespace gsrad {

template <int K>
__device__ __forceinline__ void sh_eval(float x, float y, float z, float (&Y)[K]) {
    Y[0] = 0.282094791773878f;
    if constexpr (K > 1) {
        Y[1] = 0.488602511902920f * y;
        Y[2] = 0.488602511902920f * z;
        Y[3] = 0.488602511902920f * x;
    }
    if constexpr (K > 4) {
        const float xx = x * x, yy = y * y, zz = z * z;
        Y[4] = 1.092548430592079f * (x * y);
        Y[5] = 1.092548430592079f * (y * z);
        Y[6] = 0.315391565252520f * (3.0f * zz - 1.0f);
        Y[7] = 1.092548430592079f * (x * z);
        Y[8] = 0.546274215296040f * (xx - yy);
        if constexpr (K > 9) {
            Y[9] = 0.590043589926644f * (y * (3.0f * xx - yy));
            Y[10] = 2.890611442640554f * (x * y * z);
            Y[11] = 0.457045799464466f * (y * (5.0f * zz - 1.0f));
            Y[12] = 0.373176332590115f * (z * (5.0f * zz - 3.0f));
            Y[13] = 0.457045799464466f * (x * (5.0f * zz - 1.0f));
            Y[14] = 1.445305721320277f * (z * (xx - yy));
            Y[15] = 0.590043589926644f * (x * (xx - 3.0f * yy));
        }
    }
}

// degree l and order m of coefficient a
__host__ __device__ constexpr int sh_l(int a) { return a < 1 ? 0 : a < 4 ? 1 : a < 9 ? 2 : 3; }
__host__ __device__ constexpr int sh_m(int a) { return a - sh_l(a) * sh_l(a) - sh_l(a); }

}  // namespace gsrad
