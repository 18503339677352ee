// Grid sizes of the batched (heterogeneous) form: the persistent kernel
// and the tuner's pass variants are compiled for these cubic lengths.
#pragma once

namespace fft3d {

#define FFT3D_FOR_EACH_MANY_SIZE(X)                                            \
    X(24) X(30) X(32) X(36) X(40) X(48) X(50) X(60) X(64) X(72) X(80) X(90)    \
    X(96) X(100) X(120) X(128)

constexpr bool many_size_supported(int n)
{
#define FFT3D_MANY_EQ(m) n == m ||
    return FFT3D_FOR_EACH_MANY_SIZE(FFT3D_MANY_EQ) false;
#undef FFT3D_MANY_EQ
}

}  // namespace fft3d
