// complex64 instantiation of the FFT passes (inner solves of the
// mixed-precision form).
#include "fft_passes.hpp"

namespace fwi {
template void launch_vie<float>(const Geo&, const Twiddles&, int, const c64*, const c64*, const int*, const c64*,
                                const c64*, const int*, c64*, c64*, c64*, const c64*, int, hipStream_t,
                                c64*, double*, VieDots*, const XUpdate*);
template void launch_vie_rows<float>(const Geo&, const Twiddles&, int, const c64*, const int*, const c64*, c64*,
                                     hipStream_t, const XUpdate*, const OrthIn*, const StartIn*, c64*);
template void launch_vie_tail<float>(const Geo&, const Twiddles&, int, const c64*, const c64*, const int*,
                                     const c64*, const int*, c64*, c64*, c64*, const c64*, int, hipStream_t, c64*,
                                     double*, VieDots*);
template void launch_fft_padded<float>(const Geo&, const Twiddles&, const c64*, c64*, c64*, hipStream_t);
}  // namespace fwi
