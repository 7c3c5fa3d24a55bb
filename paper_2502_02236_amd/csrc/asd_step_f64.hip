// FP64 instantiation of the Heun step kernels.  Built with -ffp-contract=off:
// every FP64 operation rounds as written (IEEE round-to-nearest), in the
// fixed order of asd_step.inc.
#include "asd_step.inc"
#include "asd_fused.inc"
#include "asd_fused_l10.inc"

namespace asd {

int launch_plain_step_f64(const StepArgs<double> &a, int n_blocks, void *stream)
{
    return launch_plain<double>(a, n_blocks, stream);
}

int launch_fused_step_f64(const StepArgs<double> &a, int n_blocks, void *stream)
{
    if (a.lattice == ASD_L10) return launch_fused_l10<double>(a, n_blocks, stream);
    return launch_fused<double>(a, n_blocks, stream);
}

int launch_mc_sweep_f64(const MCArgs<double> &a, int n_tiles, void *stream)
{
    return launch_mc<double>(a, n_tiles, stream);
}

int launch_energy_f64(const EnergyArgs<double> &e, int n_tiles, void *stream)
{
    hipLaunchKernelGGL(k_energy<double>, dim3(n_tiles), dim3(kPlainTile), 0, (hipStream_t)stream, e);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace asd
