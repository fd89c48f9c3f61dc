"""Error measures used by the tests and the benchmark report.

Elementwise |y|-relative error is unbounded for any floating-point sum under
cancellation, so results are gated on the summation forward-error form
e_i = |yhat_i - y_i| / max(sum_r |x_r,i|, tau)   (Higham, Accuracy and
Stability of Numerical Algorithms, 2nd ed., ch. 4).
"""
import numpy as np

FP32_TINY = np.float64(np.finfo(np.float32).tiny)


def normalized_error(yhat, yref, abs_sum, tau=FP32_TINY):
    yhat = np.asarray(yhat, np.float64)
    yref = np.asarray(yref, np.float64)
    den = np.maximum(np.asarray(abs_sum, np.float64), tau)
    return np.abs(yhat - yref) / den


def error_report(yhat, yref, abs_sum, tau=FP32_TINY):
    e = normalized_error(yhat, yref, abs_sum, tau)
    yref = np.asarray(yref, np.float64)
    d = np.asarray(yhat, np.float64) - yref
    nrm = float(np.linalg.norm(yref))
    rel = np.abs(d) / np.maximum(np.abs(yref), tau)
    return {
        "max_norm_err": float(e.max()) if e.size else 0.0,
        "normwise_rel": float(np.linalg.norm(d) / nrm) if nrm > 0 else 0.0,
        "p999_rel": float(np.quantile(rel, 0.999)) if rel.size else 0.0,
    }
