"""Measured parity errors of the GPU tests, printed at the end of the run
(``record`` from a test; the summary hook lives in conftest.py), so each bar
in a test can be read next to the error it actually allows."""
RECORDS = []


def record(name, err, bar):
    """Note the largest error `err` a test measured against its bar."""
    RECORDS.append((str(name), float(err), float(bar)))
    return err


def allclose(name, got, ref, rtol, atol=0.0):
    """np.testing.assert_allclose(got, ref, rtol, atol), with the largest
    |got - ref| / (atol + rtol |ref|) recorded against its bar of 1 (NaN in
    the same places on both sides counts as equal, as the assertion takes it)."""
    import numpy as np

    g = np.asarray(got, dtype=float)
    r = np.asarray(ref, dtype=float)
    lim = atol + rtol * np.abs(r)
    with np.errstate(divide="ignore", invalid="ignore"):
        q = np.where(lim > 0, np.abs(g - r) / lim, np.where(g == r, 0.0, np.inf))
    q = np.where(np.isnan(g) & np.isnan(r), 0.0, q)
    worst = float(np.nanmax(q)) if q.size and not np.all(np.isnan(q)) else 0.0
    record(f"{name} (error / bar)", worst, 1.0)
    np.testing.assert_allclose(g, r, rtol=rtol, atol=atol, err_msg=name)
