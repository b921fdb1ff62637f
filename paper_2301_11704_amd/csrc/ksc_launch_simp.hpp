// Launchers of the implicit-in-s step (ksc_simp.hip): banded solves along s,
// between the host runtime and the kernel translation unit.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "ksc_tile.hpp"

namespace ksc {

// Rows of one chain handled by one thread at most (the chunk length bound, 8
// or 16: a template parameter of the kernel).  A chain of n rows is cut into
// P <= 256 chunks, so n <= 256 * 16.
constexpr int kSimpChunkMax = 16;
constexpr int kSimpMaxChunks = 256;
constexpr int kSimpLog2Threads = 9;
constexpr int kSimpThreads = 1 << kSimpLog2Threads;

// One workgroup: the rows j = 1 + parity, 3 + parity, ... <= n_s - 2 of one
// curve, for the mode columns col0 .. col0 + CW - 1, with P = 2^log2p chunks
// and CW = kSimpThreads / P columns.
struct SimpBlock {
  int curve;
  int parity;
  int col0;
  int log2p;
};

template <typename T>
struct SimpArgs {
  const T* __restrict__ in;        // state
  const T* __restrict__ grad;      // Euclidean gradient of J2 of `in` (state layout)
  T* __restrict__ out;             // next state
  const CurveDev* __restrict__ curves;
  const T* __restrict__ cs;        // per row: g_j / (2 dsigma), 0 on the end rows
  const T* __restrict__ wlT;       // per row: 2 w_j L
  const T* __restrict__ A;         // per mode: A_k = q_k^2 - q_k^4
  const SimpBlock* __restrict__ blocks;
  const uint8_t* __restrict__ active;  // nullable
  T dtau;
  T beta;                          // heavy-ball momentum: out += beta (in - out on entry); 0: off
  const uint8_t* __restrict__ rose;  // per curve: 1 restarts the momentum (the cost just rose)
  int odd;                         // rows of K reals (modes 1..K) instead of K+1 complex
};

// chunk: the chunk length bound the solve table was built for (8 or 16).
hipError_t launch_simp_f32(int chunk, int n_blocks, hipStream_t s, const SimpArgs<float>& a);
hipError_t launch_simp_f64(int chunk, int n_blocks, hipStream_t s, const SimpArgs<double>& a);

}  // namespace ksc
