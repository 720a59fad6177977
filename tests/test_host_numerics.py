"""Host-side checks of numeric facts the kernels rely on (no device)."""
import numpy as np
import pytest


@pytest.mark.parametrize("dtype,big", [(np.float32, 1e18), (np.float64, 1e110)])
def test_force_row_sentinel_terms_are_exactly_zero(dtype, big):
    """The force adjoint stages a solute cell of a kept x-row at x = BIG with
    zero field.  With any atom inside the box (|d| at most a few nm) every
    term of that pair must come out exactly zero in the working precision:
    r^2 stays finite, r^-3 underflows, and the field products are zeros.
    The pair's operations are replayed here in their order."""
    rng = np.random.default_rng(3)
    one = dtype(1)
    for _ in range(200):
        ax, dy, dz = (dtype(v) for v in rng.uniform(-8, 8, 3))
        c1, c2, k3 = (dtype(v) for v in rng.uniform(1e-6, 10, 3))
        ex = ey = ez = dtype(0)
        with np.errstate(under="ignore"):
            dx = dtype(big) - ax
            ryz = dy * dy + dz * dz
            r2 = dx * dx + ryz
            assert np.isfinite(r2)
            ir = one / np.sqrt(r2)
            ir2 = ir * ir
            ir3 = ir2 * ir
            ir5 = ir3 * ir2
            ir6 = ir3 * ir3
            ed = ex * dx + ey * dy + ez * dz
            lj3 = ir3 * (c1 * ir6 - c2)
            coef = ir5 * (lj3 - k3 * ed)
            terms = [coef * dx, coef, ir3 * ex, ir3 * ey, ir3 * ez]
        assert ir5 == 0 and ir6 == 0 and ed == 0
        assert all(t == 0 for t in terms), terms
