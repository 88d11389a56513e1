// Real spherical harmonics storage (Sect. 4.5): for linear algebra the
// coefficient vector holds r_lm for every -l <= m <= l as real numbers, with
// r_l,-m in the slot of Im a_lm.  With R_l0 = Y_l0, R_lm = sqrt(2) Re Y_lm and
// R_l,-m = sqrt(2) Im Y_lm (m > 0) the complex coefficients of the same real
// field are a_l0 = r_l0 and a_lm = (r_lm - i r_l,-m) / sqrt(2).  These kernels
// convert between the two storages around the Legendre steps.
#include <hip/hip_runtime.h>

#include "sht_internal.h"

namespace sht {

// One thread per (m, l), looping over the rows (transform, component).
// TO_COMPLEX: r -> a; else a -> r (in place allowed: each element is read and
// written by the same thread).
template <bool TO_COMPLEX>
__global__ __launch_bounds__(256) void k_real_harm(const double2 *in, double2 *out, int lmax, int nrows,
                                                   int64_t nalm)
{
    const int m = blockIdx.y;
    const int l = m + (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (l > lmax) return;
    const int64_t idx = (int64_t)m * (2 * (int64_t)lmax + 1 - m) / 2 + l;
    const double s = TO_COMPLEX ? 0.70710678118654752440 : 1.41421356237309504880;   // 1/sqrt 2, sqrt 2
    for (int row = 0; row < nrows; ++row) {
        const double2 v = in[(int64_t)row * nalm + idx];
        out[(int64_t)row * nalm + idx] = m == 0 ? make_double2(v.x, 0.0) : make_double2(s * v.x, -s * v.y);
    }
}

int launch_real_harm(const Plan &p, const double *in, double *out, int ncomp, bool to_complex, hipStream_t s)
{
    const dim3 grid((unsigned)((p.lmax + 1 + 255) / 256), (unsigned)(p.mmax + 1));
    const int nrows = p.ntrans * ncomp;
    const double2 *i2 = reinterpret_cast<const double2 *>(in);
    double2 *o2 = reinterpret_cast<double2 *>(out);
    if (to_complex) hipLaunchKernelGGL(k_real_harm<true>, grid, dim3(256), 0, s, i2, o2, p.lmax, nrows, p.nalm);
    else hipLaunchKernelGGL(k_real_harm<false>, grid, dim3(256), 0, s, i2, o2, p.lmax, nrows, p.nalm);
    return check_hip(hipGetLastError(), "real harmonics launch");
}

}  // namespace sht
