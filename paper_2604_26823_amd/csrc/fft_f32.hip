// FP32 instantiations of the FFT passes.
#include "fft_impl.h"

namespace ic {
template void fft_r2c_z<float>(const FftArgs<float>&, const float*, float, const float*, float,
                               cx<float>*, const float*);
template void fft_c2r_z<float>(const FftArgs<float>&, const cx<float>*, float*, float,
                               const float*, float);
template void fft_y<float>(const FftArgs<float>&, cx<float>*, bool);
template bool fft_zy_fused<float>(int);
template void fft_r2c_zy<float>(const FftArgs<float>&, const float*, float, const float*, float,
                                cx<float>*, const float*);
template void fft_c2r_yz<float>(const FftArgs<float>&, const cx<float>*, float*);
template void fft_x<float>(const FftArgs<float>&, const cx<float>*, cx<float>*, bool, float);
template void spectrum_pack<float>(const FftArgs<float>&, const cx<float>*, cx<float>*);
template void spectrum_unpack<float>(const FftArgs<float>&, const cx<float>*, cx<float>*);
template void fft_x_scatter<float>(const FftArgs<float>&, const cx<float>*, cx<float>* const*,
                                   const MulSpec*, int);
template void fft_x_gather<float>(const FftArgs<float>&, const cx<float>* const*,
                                  const MulSpec*, int, cx<float>*);
}  // namespace ic
