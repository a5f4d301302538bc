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
// In-place forward transform of data[n][n][n] on stream st.  Pruning (a
// half-extent e > 0 names the wrapped centred cube m < e or m >= n - e of
// every axis; e = 0 or 2e >= n means the whole axis):
//  * e_in: the input is zero outside that cube (its values there are not
//    read), so lines of zeros are skipped and each line is read only in the
//    band;
//  * e_out: only outputs inside that cube are wanted; the lines that cannot
//    reach them are skipped, each line is written only in the band, and the
//    rest of the array is left undefined.
hsd_status fft3d_forward(hipStream_t st, const FftPlan &p, double2 *data, int e_in = 0, int e_out = 0);
// Bytes the three passes of fft3d_forward(n, e_in, e_out) read and write:
// each pass reads its lines in the input band and writes them in the output
// band, 16 bytes per complex value.
double fft3d_bytes(int n, int e_in, int e_out);

} // namespace hsd
