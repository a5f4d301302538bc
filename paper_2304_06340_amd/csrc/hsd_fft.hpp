// hsd_fft.hpp -- plan of the cubic 3-D FFT (hsd_fft.hip).
#pragma once

#include <vector>

#include "hsd_internal.hpp"

namespace hsd {

struct FftPlan {
    int n = 0;
    std::vector<int> stages;   // radices, product = n
    DevBuf tw;                 // exp(-2 pi i k / n), k < n
    DevBuf plan;               // stages on the device
    hsd_status init(hsd_ctx *ctx, int n);
};

bool fft_size_ok(int n);
int fft_next_size(int n);
// In-place forward transform of data[n][n][n] on stream st.
hsd_status fft3d_forward(hipStream_t st, const FftPlan &p, double2 *data);

} // namespace hsd
