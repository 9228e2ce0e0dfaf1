"""MI355X (gfx950) implementation of the iterative full-scale-approximation
Gaussian-process path of Gyger, Furrer & Sigrist (arXiv 2405.14492):
block PCG with the FITC preconditioner, SLQ log-determinants, stochastic
gradients and simulation-based predictive variances, behind the C ABI of
include/fsa.h (libfsa.so)."""
from .fsa import (CV_NONE, CV_ONE, CV_OPT, CV_OPT_PRINTED, EXPONENTIAL, FP64, FSA, MATERN32, MIXED_BF16A, MIXED_FP32,
                  FsaError, NotConverged, fsa_apply, fsa_build, fsa_build_dev, fsa_destroy, fsa_export_csr,
                  fsa_export_diag, fsa_export_lanczos, fsa_grad, fsa_nll_grad, fsa_nnz, fsa_predict_var, fsa_scores,
                  make_options)

__all__ = ["FSA", "FsaError", "NotConverged", "EXPONENTIAL", "MATERN32", "FP64", "MIXED_FP32", "MIXED_BF16A", "CV_NONE",
           "CV_ONE", "CV_OPT", "CV_OPT_PRINTED", "fsa_build", "fsa_build_dev", "fsa_nll_grad", "fsa_grad",
           "fsa_predict_var", "fsa_destroy", "fsa_export_csr", "fsa_export_diag", "fsa_export_lanczos", "fsa_apply",
           "fsa_nnz", "fsa_scores", "make_options"]
