"""MI355X-native fermion-matrix solve for Hybrid Monte Carlo of the Hubbard model
on the honeycomb lattice: HIP kernels for CDNA4 behind the C ABI of include/hub.h,
with a thin Python binding (torch supplies device memory and streams only).
"""
from .binding import (  # noqa: F401
    HUB_CG_FP64, HUB_FGMRES_MIXED, HUB_MAX_BATCH, Context, HubError, PseudofermionAction, default_opts,
    hub_action, hub_apply_M, hub_apply_Mdag, hub_apply_normal, hub_force, hub_hasenbusch_force,
    hub_hasenbusch_heatbath, hub_hasenbusch_masses, hub_hmc_trajectory, hub_hmc_trajectories, hub_solve_multishift, hub_md_schedule, hmc_params, hub_poll, hub_profile_enable,
    hub_profile_read, hub_solve, hub_submit,
    lattice, load,
)
