// Dense stage kernels and host sequencing (first part: exact-core densification).
#include "dense.hpp"

namespace tts {

namespace {

constexpr int NT = 256;

// core[(rho) * beta_k + col] = N_k[rho, col]; one thread per column of N_k.
__global__ __launch_bounds__(NT) void k_densify(const int64_t* __restrict__ colptr, const int32_t* __restrict__ row,
                                                const double* __restrict__ val, uint32_t ncols,
                                                double* __restrict__ core) {
  const uint32_t c = blockIdx.x * NT + threadIdx.x;
  if (c >= ncols) return;
  for (int64_t e = colptr[c]; e < colptr[c + 1]; ++e)
    core[static_cast<int64_t>(row[e]) * ncols + c] = val[e];
}

}  // namespace

void densify_exact_cores(Allocator& al, const RoundInput& in, std::vector<DBuf<char>>& cores, hipStream_t s) {
  const int d = in.d;
  double total = 0.0;
  for (int k = 1; k <= d; ++k) total += static_cast<double>(in.betas[k - 1]) * in.dims[k - 1] * in.betas[k];
  cores.clear();
  if (total > static_cast<double>(1ull << 28)) return;  // too large to densify; levels stay available
  for (int k = 1; k <= d; ++k) {
    const size_t n = static_cast<size_t>(in.betas[k - 1]) * in.dims[k - 1] * in.betas[k];
    DBuf<char> c(&al, n * sizeof(double));
    if (k < d) {
      TTS_HIP(hipMemsetAsync(c.get(), 0, n * sizeof(double), s));
      const uint32_t ncols = static_cast<uint32_t>(in.betas[k]);
      k_densify<<<grid_for(ncols, NT), NT, 0, s>>>(in.n_colptr[k - 1], in.n_row[k - 1], in.n_val[k - 1], ncols,
                                                   reinterpret_cast<double*>(c.get()));
      TTS_LAUNCH_CHECK();
    } else {
      TTS_HIP(hipMemcpyAsync(c.get(), in.last_core, n * sizeof(double), hipMemcpyDeviceToDevice, s));
    }
    cores.push_back(std::move(c));
  }
}

}  // namespace tts
