// Stand-ins for the library's device entry points, linked with the host
// runtime (crkfr_host.hip) into a CPU-only sanitizer build: every launch
// reports "no kernel", so only host code runs (the Fourier CFL analysis, the
// reference element, argument checks and their error paths).
#include "../../paper_2502_07517_amd/csrc/crkfr_launch.hpp"
#include "../../paper_2502_07517_amd/csrc/crkfr_internal.hpp"

namespace crkfr {

#define CRKFR_STUB_EQ(name)                                                                                   \
    int name##_step_f64(int, bool, int, const StepArgs<double>&, hipStream_t) { return -1; }                   \
    int name##_step_f32(int, bool, int, const StepArgs<float>&, hipStream_t) { return -1; }                    \
    int name##_io_f64(int, int, const IoArgs<double>&, hipStream_t) { return -1; }                             \
    int name##_io_f32(int, int, const IoArgs<float>&, hipStream_t) { return -1; }                              \
    int name##_batch_f64(int, bool, int, const StepArgs<double>*, const int2*, int, int, hipStream_t) { return -1; } \
    int name##_batch_f32(int, bool, int, const StepArgs<float>*, const int2*, int, int, hipStream_t) { return -1; }  \
    int name##_geometry(int, int*, int*, int*) { return -1; }                                                  \
    int name##_tile_shape(int, int, int*, int*) { return -1; }

CRKFR_STUB_EQ(linadv1d)
CRKFR_STUB_EQ(euler1d)
CRKFR_STUB_EQ(euler2d)
CRKFR_STUB_EQ(tenmom2d)
CRKFR_STUB_EQ(burgers1d)
CRKFR_STUB_EQ(tenmom1d)

const float* mlp_device_params(const crkfr_mlp*) { return nullptr; }
int mlp_inputs(const crkfr_mlp*) { return 0; }
int mlp_hidden(const crkfr_mlp*) { return 0; }

}  // namespace crkfr
