// FP64 instantiations of the FFT passes.
#include "fft_impl.h"

namespace ic {
template void fft_r2c_z<double>(const FftArgs<double>&, const double*, double, const double*, double,
                               cx<double>*, const double*);
template void fft_c2r_z<double>(const FftArgs<double>&, const cx<double>*, double*, double,
                               const double*, double);
template void fft_y<double>(const FftArgs<double>&, cx<double>*, bool);
template bool fft_zy_fused<double>(int);
template void fft_r2c_zy<double>(const FftArgs<double>&, const double*, double, const double*, double,
                                 cx<double>*, const double*);
template void fft_c2r_yz<double>(const FftArgs<double>&, const cx<double>*, double*);
template void fft_x<double>(const FftArgs<double>&, const cx<double>*, cx<double>*, bool, double);
template void spectrum_pack<double>(const FftArgs<double>&, const cx<double>*, cx<double>*);
template void spectrum_unpack<double>(const FftArgs<double>&, const cx<double>*, cx<double>*);
template void fft_x_scatter<double>(const FftArgs<double>&, const cx<double>*, cx<double>* const*,
                                   const MulSpec*, int);
template void fft_x_gather<double>(const FftArgs<double>&, const cx<double>* const*,
                                  const MulSpec*, int, cx<double>*);
}  // namespace ic
