"""Shared parity assertions for the GPU tests (imported by the test modules)."""
from oracle import metrics as M


def assert_xhat(got, ref, tol, what=""):
    """Detected symbols [..., n_sc, n_ue] against the oracle: whole-tensor NRMSE <= tol, and every
    element and every subcarrier's RMS error within 10 tol of the reference RMS, so that a wrong
    block of subcarriers or a wrong tail path cannot hide in the aggregate."""
    e = M.xhat_errors(got, ref)
    msg = f"{what} nrmse {e['nrmse']:.3e} max-rel {e['max_rel']:.3e} worst-sc {e['worst_sc']:.3e} (tol {tol:g})"
    print(msg)
    assert e["nrmse"] <= tol and e["max_rel"] <= 10 * tol and e["worst_sc"] <= 10 * tol, msg
    return e
