// complex128 instantiation of the FFT passes (plain FP64 path, FP64 residuals,
// Green spectra).
#define FWI_FFT_WITH_FULL
#include "fft_passes.hpp"

namespace fwi {
template void launch_vie<double>(const Geo&, const Twiddles&, int, const c128*, const c128*, const int*, const c128*,
                                 const c128*, const int*, c128*, c128*, c128*, const c128*, int, hipStream_t,
                                 c64*, double*, VieDots*, const XUpdate*);
template void launch_vie_rows<double>(const Geo&, const Twiddles&, int, const c128*, const int*, const c128*, c128*,
                                     hipStream_t, const XUpdate*, const OrthIn*, const StartIn*, c128*);
template void launch_vie_tail<double>(const Geo&, const Twiddles&, int, const c128*, const c128*, const int*,
                                     const c128*, const int*, c128*, c128*, c128*, const c128*, int, hipStream_t, c64*,
                                     double*, VieDots*);
template void launch_fft_padded<double>(const Geo&, const Twiddles&, const c128*, c128*, c128*, hipStream_t);
}  // namespace fwi
