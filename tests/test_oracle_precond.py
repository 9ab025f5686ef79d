"""Pins of the learned block-Jacobi correction's reference (no GPU).

- zero output layer gives exactly the block-Jacobi preconditioner;
- the normalised coupling E_i equals the diagonal block of the square of
  the densely normalised matrix, minus I;
- the loss at C = I is the mean trace of E, its C-gradient vanishes at the
  closed-form minimiser C_i = chol((I + E_i)^-1) and the loss grows away
  from it;
- the hand-written parameter gradient matches central differences;
- relabelling the cameras permutes the outputs;
- the PCG iteration counter agrees with the C oracle's PCG.
"""
import numpy as np
import pytest

from oracle import oracle as O
from oracle import precond_oracle as G
from synth.scenes import make_scene


@pytest.fixture(scope="module")
def system():
    s = make_scene(1, n_cams=40, n_pts=1500, seed=2)
    o = O.Oracle.from_scene(s)
    o.compute_step(rtol=1e-4, maxiter=5)
    ptr, col, S, bS = o.schur()
    return s, o, ptr, col, S, bS


def test_zero_output_is_block_jacobi(system):
    s, o, ptr, col, S, bS = system
    g = G.system_graph(ptr, col, S, s.n_cams)
    theta = G.init_params(np.random.default_rng(0))
    M = G.precond_blocks(theta, g)
    for a in range(s.n_cams):
        D = S[ptr[a]]
        assert np.abs(M[a] @ D - np.eye(9)).max() < 1e-9


def test_normalised_coupling_matches_dense(system):
    s, o, ptr, col, S, bS = system
    nc = s.n_cams
    g = G.system_graph(ptr, col, S, nc)
    A = np.zeros((9 * nc, 9 * nc))
    for a in range(nc):
        for e in range(ptr[a], ptr[a + 1]):
            b = col[e]
            A[9 * a:9 * a + 9, 9 * b:9 * b + 9] = S[e]
            if b != a:
                A[9 * b:9 * b + 9, 9 * a:9 * a + 9] = S[e].T
    Dinv = np.zeros_like(A)
    for a in range(nc):
        Dinv[9 * a:9 * a + 9, 9 * a:9 * a + 9] = np.linalg.inv(np.linalg.cholesky(A[9 * a:9 * a + 9, 9 * a:9 * a + 9]))
    An = Dinv @ A @ Dinv.T
    A2 = An @ An
    for a in range(nc):
        Eref = A2[9 * a:9 * a + 9, 9 * a:9 * a + 9] - np.eye(9)
        assert np.abs(g["E"][a] - Eref).max() <= 1e-9 * max(1.0, np.abs(Eref).max())


def test_loss_minimiser_and_value_at_identity(system):
    s, o, ptr, col, S, bS = system
    g = G.system_graph(ptr, col, S, s.n_cams)
    n = s.n_cams
    I = np.tile(np.eye(9), (n, 1, 1))
    assert abs(G.loss_from_C(I, g) - np.mean(np.trace(g["E"], axis1=1, axis2=2))) < 1e-10
    Cs = np.linalg.cholesky(np.linalg.inv(np.eye(9) + g["E"]))
    assert np.abs(G.dloss_dC(Cs, g)).max() < 1e-10
    l0 = G.loss_from_C(Cs, g)
    rng = np.random.default_rng(1)
    for _ in range(5):
        D = np.tril(rng.normal(size=Cs.shape)) * 1e-3
        assert G.loss_from_C(Cs + D, g) > l0


def test_parameter_gradient_matches_central_differences(system):
    s, o, ptr, col, S, bS = system
    g = G.system_graph(ptr, col, S, s.n_cams)
    rng = np.random.default_rng(3)
    theta = G.init_params(rng)
    d = G.unpack(theta)
    d["W_out"][:] = rng.normal(size=d["W_out"].shape) * 0.05
    d["b_out"][:] = rng.normal(size=d["b_out"].shape) * 0.05
    theta = G.pack(d)
    gr = G.grad(theta, g)
    idx = rng.choice(theta.size, 80, replace=False)
    idx = np.concatenate([idx, np.arange(theta.size - 45, theta.size)[:5]])
    h = 1e-6
    for i in idx:
        e = np.zeros_like(theta)
        e[i] = h
        fd = (G.loss(theta + e, g) - G.loss(theta - e, g)) / (2 * h)
        assert abs(fd - gr[i]) <= 1e-6 * max(1.0, abs(fd)) + 1e-7 * np.abs(gr).max(), (i, fd, gr[i])


def test_relabelling_cameras_permutes_outputs(system):
    s, o, ptr, col, S, bS = system
    g = G.system_graph(ptr, col, S, s.n_cams)
    rng = np.random.default_rng(4)
    theta = G.init_params(rng)
    d = G.unpack(theta)
    d["W_out"][:] = rng.normal(size=d["W_out"].shape) * 0.1
    theta = G.pack(d)
    perm = rng.permutation(s.n_cams)
    gp = dict(g)
    gp["X"] = g["X"][perm]
    gp["P"] = g["P"][np.ix_(perm, perm)]
    o1, _ = G.forward(theta, g)
    o2, _ = G.forward(theta, gp)
    assert np.abs(o2 - o1[perm]).max() < 1e-12


def test_pcg_counter_matches_c_oracle(system):
    s, o, ptr, col, S, bS = system
    g = G.system_graph(ptr, col, S, s.n_cams)
    M = np.linalg.inv(g["diag"])
    k = G.pcg_iterations(ptr, col, S, bS, M, 1e-6, 2000)
    info = o.compute_step(rtol=1e-6, maxiter=2000)
    assert k == info["cg_iters"]


def test_bf16_rounding_by_definition():
    """Round-to-nearest-even onto 8 significant bits: exact values stay,
    halfway cases go to the even neighbour, others to the nearest."""
    one = 1.0
    ulp = 2.0 ** -7                       # spacing of bfloat16 in [1, 2)
    cases = [(one, one), (one + ulp, one + ulp), (one + ulp / 2, one),
             (one + 3 * ulp / 2, one + 2 * ulp), (one + ulp / 2 + 2 ** -20, one + ulp),
             (-3.0, -3.0), (0.0, 0.0), (2.0 ** -30 * 1.75, 2.0 ** -30 * 1.75)]
    for x, want in cases:
        assert G.bf16(x) == want, (x, G.bf16(x), want)


def test_bf16_inference_rounds_message_layer_operands_only(system):
    """The rounded network keeps the input layer exact; a message layer whose
    operands are already on the bfloat16 grid is the exact one (W_in = 0 and
    b_in on the grid make h0 representable, W_m = 0 drops the messages), and
    moving its weights off the grid changes it."""
    s, o, ptr, col, S, bS = system
    g = G.system_graph(ptr, col, S, s.n_cams)
    rng = np.random.default_rng(5)
    d = G.unpack(G.init_params(rng))
    o_exact, c_exact = G.forward(G.pack(d), g)
    o_b, c_b = G.forward(G.pack(d), g, bf16_inference=True)
    np.testing.assert_array_equal(c_b["z"][0], c_exact["z"][0])
    d["W_in"][:] = 0.0
    d["b_in"][:] = G.bf16(rng.normal(size=d["b_in"].shape))
    d["W_s0"][:] = G.bf16(d["W_s0"])
    d["W_m0"][:] = 0.0
    _, c_exact = G.forward(G.pack(d), g)
    _, c_b = G.forward(G.pack(d), g, bf16_inference=True)
    np.testing.assert_array_equal(c_b["z"][1], c_exact["z"][1])
    d["W_s0"][:] *= 1.0 + 2.0 ** -10      # off the grid: rounded back in the inference form
    _, c_exact = G.forward(G.pack(d), g)
    _, c_b = G.forward(G.pack(d), g, bf16_inference=True)
    assert not np.array_equal(c_b["z"][1], c_exact["z"][1])
