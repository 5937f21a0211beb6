"""MI355X library for the online solve of the HR DD NM-ROM (arXiv 2305.15163):
HIP kernels for gfx950 behind a C ABI (include/ddrom.h), with a thin ctypes binding."""
from .ddrom import (PREC_FP32_DECODER, PREC_FP64, STATUS, AETrainer, Model, Proposal, ProposalTrainer, Workspace, ae_decode_hr,
                    autotune_tiles, model_desc,
                    ae_jacobian_hr, ae_jacobian_hr_noalloc, dd_fom_residual, decode_states, gn_blocks, lib, mlp_proposal, opts,
                    pack_mlp_params, relative_error, rom_solve_batch, rom_solve_multi, rom_solve_warm, sqp_step, time_kernels,
                    unpack_mlp_params, ae_pack, ae_unpack)

__all__ = ["PREC_FP32_DECODER", "PREC_FP64", "STATUS", "AETrainer", "Model", "Proposal", "ProposalTrainer", "Workspace",
           "ae_decode_hr", "ae_jacobian_hr", "ae_jacobian_hr_noalloc", "autotune_tiles", "model_desc", "dd_fom_residual", "decode_states", "gn_blocks", "lib",
           "mlp_proposal", "opts", "pack_mlp_params", "relative_error", "rom_solve_batch", "rom_solve_multi", "rom_solve_warm",
           "sqp_step", "time_kernels", "unpack_mlp_params", "ae_pack", "ae_unpack"]
