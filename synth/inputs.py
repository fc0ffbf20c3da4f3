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


def halo_net_weights(seed):
    """Seeded weights of the two-network halo model (untrained): the position network
    81 -> 50 -> 30 -> 1 and the mass network 3 -> 20 -> 10 -> 1, float32 row-major
    [out][in]. Hidden weights ~ N(0, 2 / fan_in), hidden biases ~ N(0, 0.01^2); the mass
    network's output layer is scaled by 0.1 with bias 1, so that its (linear) output stays
    near 1 and the modelled mass stays positive."""
    r = _rng(seed)

    def layer(n_out, n_in, scale=None):
        s = np.sqrt(2.0 / n_in) if scale is None else scale
        return (r.standard_normal((n_out, n_in)) * s).astype(np.float32), \
            (r.standard_normal(n_out) * 0.01).astype(np.float32)

    nnp, nnm = {}, {}
    nnp["W1"], nnp["b1"] = layer(50, 81)
    nnp["W2"], nnp["b2"] = layer(30, 50)
    nnp["W3"], nnp["b3"] = layer(1, 30)
    nnm["W1"], nnm["b1"] = layer(20, 3)
    nnm["W2"], nnm["b2"] = layer(10, 20)
    nnm["W3"], b = layer(1, 10, scale=0.1 * np.sqrt(2.0 / 10))
    nnm["b3"] = (b + 1.0).astype(np.float32)
    return {"nnp": {k: np.ascontiguousarray(v) for k, v in nnp.items()},
            "nnm": {k: np.ascontiguousarray(v) for k, v in nnm.items()}}
