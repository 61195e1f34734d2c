"""Error of every intermediate of the path against the FP64 oracle, on both
precisions, for the Matern nu = 1 workload (256^2 grid, the ladder's 768
torus, 1000 uniform stations, 6 x 6 windows, nugget 0.1, 8 realizations):
sqrt(lambda), the window weights and gamma, the unconditional draws y_r, the
synthetic data z*_r, the coefficients alpha_r = A^{-1}(z - z*_r) and the
conditional fields v_r.  z*_r is not exposed by the ABI; it is recovered from
the library's coefficients as z - A alpha_r with the oracle's A.  Prints one
line per precision (run with -s to see it) and holds each error to its bound."""
import numpy as np
import pytest

from oracle import kriging
from oracle.covariance import Cov as OCov
from oracle.pipeline import Grid as OGrid
from oracle.pipeline import conditional_simulation, draw_observations, setup
from paper_2109_11044_amd import cesim, workloads

pytestmark = pytest.mark.gpu

# precision -> bound per intermediate (relative to the largest reference
# value, relative RMS per field for y and v, absolute for gamma)
BOUNDS = {
    "fp64": dict(lam=1e-12, w=1e-9, gamma=1e-12, y=1e-12, zstar=1e-9, alpha=1e-9, v=1e-10),
    "mixed": dict(lam=1e-12, w=1e-9, gamma=1e-12, y=1e-6, zstar=1e-5, alpha=1e-4, v=1e-4),
}


def rel_rms(a, b):
    a = np.asarray(a, dtype=np.float64).reshape(a.shape[0], -1)
    b = np.asarray(b, dtype=np.float64).reshape(b.shape[0], -1)
    return float(np.max(np.sqrt(np.mean((a - b) ** 2, axis=1) / np.mean(b ** 2, axis=1))))


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_error_of_every_intermediate(prec):
    wl = workloads.C2
    R, seed = 8, 2
    xy = wl.obs_xy()
    ocov = OCov(wl.nu, wl.sigma2, wl.range)
    og = OGrid.unit_square(wl.m)
    z = draw_observations(xy, ocov, wl.tau2, seed=0)
    with cesim.Context(cesim.make_cov(wl.nu, wl.sigma2, wl.range), cesim.unit_square_grid(wl.m),
                       prec) as ctx:
        t = ctx.info()["t1"]
        s = ctx.spectrum().cpu().numpy()
        ctx.offgrid(xy, wl.k)
        _, w, gm = (a.cpu().numpy() for a in ctx.weights())
        f = ctx.simulate(R, seed)
        y = f.cpu().numpy()
        ctx.condition(z, wl.tau2, f)
        v = f.cpu().numpy()
        alpha = ctx.coefficients().cpu().numpy()           # [R][n]
    ref = conditional_simulation(ocov, og, xy, z, wl.tau2, wl.k, seed, R, 0, t, t)
    _, _, sref, _ = setup(ocov, og, t, t)
    A = kriging.obs_matrix(xy, ocov, wl.tau2)
    zstar = z[None, :] - alpha @ A                          # A symmetric
    err = dict(
        lam=float(np.max(np.abs(s * t - sref)) / sref.max()),      # s = sqrt(lambda / t^2)
        w=float(np.max(np.abs(w - ref["W"])) / np.abs(ref["W"]).max()),
        gamma=float(np.max(np.abs(gm - ref["gamma"]))),
        y=rel_rms(y, ref["y"]),
        zstar=float(np.max(np.abs(zstar - ref["zstar"])) / np.abs(ref["zstar"]).max()),
        alpha=float(np.max(np.abs(alpha - ref["B"].T)) / np.abs(ref["B"]).max()),
        v=rel_rms(v, ref["v"]),
    )
    print(f"\nerror report {prec} (torus {t}): "
          + ", ".join(f"{k} {e:.2e}" for k, e in err.items()), flush=True)
    for k, e in err.items():
        assert e < BOUNDS[prec][k], (k, e)
