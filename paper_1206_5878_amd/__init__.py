"""MI355X-native Henon Monte Carlo step (arXiv:1206.5878, Sec. 2.1).

The hot path -- radial sort, cumulative-mass potential, pair relaxation and
orbit resampling -- runs as hand-written HIP in ``libcmc.so`` behind the C ABI
of ``include/cmc.h``.  This package holds that library, its sources, and a
thin binding with the same call names.
"""
from ._capi import (CMC_BUCKET_CAP_MAX, CMC_FP64, CMC_MIXED, CMC_MODEL_KING, CMC_MODEL_PLUMMER,
                    CMC_RNG_LFSR113, CMC_RNG_PHILOX, CMC_STEP_DEVICE,
                    CmcError, ST_BOUND, ST_DT_DEGEN, ST_DT_NOCONV,
                    ST_ESCAPER, ST_NONFINITE, ST_NUMERIC, ST_TRIAL_CAP, lib)
from . import evolve
from .cluster import (Cluster, Ensemble, Params, cmc_diagnostics, cmc_energy_correction,
                      cmc_init_model, cmc_init_plummer, cmc_orbit,
                      cmc_lfsr113, cmc_philox, cmc_potential, cmc_relax, cmc_rng_seed_lfsr113,
                      cmc_sort, cmc_step, cmc_step_noalloc, cmc_step_timed, cmc_timestep)

__all__ = ["CMC_BUCKET_CAP_MAX", "CMC_FP64", "CMC_MIXED", "CMC_MODEL_KING", "CMC_MODEL_PLUMMER",
           "CMC_RNG_LFSR113", "CMC_RNG_PHILOX", "CMC_STEP_DEVICE", "cmc_lfsr113", "cmc_rng_seed_lfsr113", "CmcError", "Cluster", "Ensemble", "evolve",
           "Params", "lib", "cmc_diagnostics", "cmc_energy_correction", "cmc_init_model", "cmc_init_plummer", "cmc_orbit", "cmc_philox", "cmc_potential", "cmc_relax",
           "cmc_sort", "cmc_step", "cmc_step_noalloc", "cmc_step_timed", "cmc_timestep", "ST_BOUND", "ST_DT_DEGEN", "ST_DT_NOCONV",
           "ST_ESCAPER", "ST_NONFINITE", "ST_NUMERIC", "ST_TRIAL_CAP"]
