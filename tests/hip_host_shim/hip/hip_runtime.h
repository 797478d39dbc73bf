// Host-only stand-in for the HIP runtime header, used by tests alone: it lets
// g++ compile the device FFT building blocks (csrc/fft.h, which need nothing
// from HIP but these two qualifiers) as plain C++ for a CPU test.
#pragma once
#define __device__
#define __forceinline__ inline
