"""CPU oracle for the tactile readout — TEST INFRASTRUCTURE ONLY.

Only the tests, the package smoke check and the CPU-baseline leg of the
benchmark import this package.  The product path (the HIP library and its
binding) never does.  The oracle shares no code with the product: it has its
own C source, its own structs and its own Python marshalling; the two meet only
in the seeded scene generator, which holds no readout arithmetic.
"""
from .oracle import (Oracle, build, run_readout, philox4x32_10, bf16_round, dense_xtalk, u01,  # noqa: F401
                     nsdf_num_params, nsdf_forward, nsdf_loss_grad, nsdf_adam, nsdf_targets, nsdf_dirderiv,
                     nsdf_forward_trace, prox_run, thermal_constants, thermal_voxel, thermal_stable, thermal_run,
                     elastomer_run, elastomer_new_state, ELASTOMER_DEFAULTS, raycast_run)
