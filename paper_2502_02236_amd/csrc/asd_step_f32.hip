// FP32 instantiation of the Heun step kernels (per-spin field and update in
// FP32; spot position and time in FP64).
#include "asd_step.inc"
#include "asd_fused.inc"
#include "asd_fused_l10.inc"

namespace asd {

int launch_plain_step_f32(const StepArgs<float> &a, int n_blocks, void *stream)
{
    return launch_plain<float>(a, n_blocks, stream);
}

int launch_fused_step_f32(const StepArgs<float> &a, int n_blocks, void *stream)
{
    if (a.lattice == ASD_L10) return launch_fused_l10<float>(a, n_blocks, stream);
    return launch_fused<float>(a, n_blocks, stream);
}

int launch_mc_sweep_f32(const MCArgs<float> &a, int n_tiles, void *stream)
{
    return launch_mc<float>(a, n_tiles, stream);
}

int launch_energy_f32(const EnergyArgs<float> &e, int n_tiles, void *stream)
{
    hipLaunchKernelGGL(k_energy<float>, dim3(n_tiles), dim3(kPlainTile), 0, (hipStream_t)stream, e);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace asd
