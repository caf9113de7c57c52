"""MI355X (gfx950) Fourier-slice Radon NUFFT: forward and adjoint Radon
transforms by gridding, behind the C ABI of include/radon.h."""
from .radon import (Batch, Plan, RadonError, Tuning, WarmStartNet, autotune, cnn_conv_test, fft_test, lib,
                    project_l1, stage_names, supported_length)

__all__ = ["Batch", "Plan", "RadonError", "Tuning", "WarmStartNet", "autotune", "cnn_conv_test", "fft_test", "lib",
           "project_l1", "stage_names", "supported_length"]
