"""FP64 CPU oracle for the rank-2 Galerkin ROM (test infrastructure only).

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
import this package.  It shares no code with the HIP library: the arithmetic
lives in ``rom_oracle.c`` (plain loops, FP64), built with gcc by
:func:`build`, and is exposed here through ctypes with numpy arrays.
"""
from .oracle import (build, lib_path, ricker, ricker_dmu, gauss1, gauss1_dmu, SOURCES, step_rank1, run_rank2,
                     energy, adjoint, num_threads, round_bf16, quantize_e4m3,
                     receivers, ensemble_stats, percentile_index, affine_operator,
                     fom_run, csr_dense, project, pod, pod_rank, run_rank2_state_bf16)

__all__ = ["build", "lib_path", "ricker", "ricker_dmu", "gauss1", "gauss1_dmu", "SOURCES", "step_rank1", "run_rank2",
           "energy", "adjoint", "num_threads", "round_bf16", "quantize_e4m3",
           "receivers", "ensemble_stats", "percentile_index", "affine_operator",
           "fom_run", "csr_dense", "project", "pod", "pod_rank", "run_rank2_state_bf16"]
