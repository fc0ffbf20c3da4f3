"""Seeded random draws (numpy PCG64). No method arithmetic lives here."""
import numpy as np


def _rng(seed):
    return np.random.Generator(np.random.PCG64(int(seed)))


def white_noise(seed, n):
    """Real white noise w(x) ~ N(0, 1) on an n^3 grid, float64, C order."""
    return _rng(seed).standard_normal((n, n, n))


def unit_normal(seed, shape):
    """Standard normal draws of arbitrary shape, float64."""
    return _rng(seed).standard_normal(shape)


def mlp_weights_raw(seed, hidden, n_in=3):
    """Standard-normal draws for a n_in -> hidden -> hidden -> 1 network.

    Returned as float64 standard normals; the caller scales them (fan-in scaling
    is a modelling choice and is applied where the weights are built).
    Layout: row-major [out][in] for weights.
    """
    r = _rng(seed)
    return {
        "W1": r.standard_normal((hidden, n_in)),
        "b1": r.standard_normal(hidden),
        "W2": r.standard_normal((hidden, hidden)),
        "b2": r.standard_normal(hidden),
        "W3": r.standard_normal((1, hidden)),
        "b3": r.standard_normal(1),
    }


def random_positions(seed, count, box):
    """Uniform positions in [0, box)^3, float64, shape (3, count)."""
    return _rng(seed).uniform(0.0, box, size=(3, count))


def random_modes_direction(seed, n):
    """Complex standard-normal array in rfft storage [n][n][n//2+1] (complex128)."""
    r = _rng(seed)
    shape = (n, n, n // 2 + 1)
    return r.standard_normal(shape) + 1j * r.standard_normal(shape)


def mlp_weights(seed, hidden, n_in=3):
    """Seeded random network weights (the halo-mass network is not trained here).

    W ~ N(0, 2 / fan_in), b ~ N(0, 0.01^2), stored as float32 row-major [out][in].
    """
    raw = mlp_weights_raw(seed, hidden, n_in)
    out = {}
    for k in ("W1", "W2", "W3"):
        out[k] = np.ascontiguousarray((raw[k] * np.sqrt(2.0 / raw[k].shape[1])).astype(np.float32))
    for k in ("b1", "b2", "b3"):
        out[k] = np.ascontiguousarray((raw[k] * 0.01).astype(np.float32))
    return out
