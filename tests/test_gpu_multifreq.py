"""GPU parity of the frequency-factored batch (eddy_solve_multifreq): systems
of three frequencies on the C1 cube (omega = 20, 50, 120) solved together,
each against the oracle's direct solve at its own frequency and against the
one-operator batched solve, at tolerance 1e-11 on the FP64 true residual
(solution bound 1e-9 as for the other complex64 solves).  The inner
process reads the factored matrix P + c(omega) Q instead of each
operator's complex64 copy, so iteration counts may differ by rounding
(within 10 %); the argument checks reject what cannot be factored."""
import numpy as np
import pytest

from synth import cube, cube_current

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

OMEGAS = (20.0, 50.0, 120.0)
STATE = {}


def setup():
    if "ops" in STATE:
        return STATE
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from oracle.assemble import assemble
    from paper_1602_03207_amd import eddy
    m = cube(8)
    nu, sig = np.array([1.0, 1.0]), np.array([0.0, 1.0])
    M = eddy.Mesh(m.xyz, m.tet, m.region, [0, 1])
    ops, sys_ = [], []
    for w in OMEGAS:
        op = eddy.Operator(M, tau=1.0, block_size=64)
        op.assemble(nu, sig, w)
        ops.append(op)
        sys_.append(assemble(m.xyz, m.tet, m.region, nu, sig, w, tau=1.0, conductor_regions=[1]))
    Js = [cube_current(m, seed) for seed in (0, 1)]
    STATE.update(m=m, M=M, ops=ops, sys=sys_, Js=Js, nu=nu, sig=sig)
    return STATE


@pytest.mark.parametrize("precision", ["mixed", "mixed16"])
def test_multifreq_matches_oracle_and_per_operator_batches(precision):
    from oracle.solve import direct
    from oracle.post import remove_v_mean
    from paper_1602_03207_amd import eddy
    S = setup()
    ops, Js = S["ops"], S["Js"]
    B = torch.stack([op.rhs_from_current(torch.from_numpy(J).cuda()) for op in ops for J in Js])
    idx = [f for f in range(len(ops)) for _ in Js]
    X, reps = eddy.solve_multifreq(ops, B, idx, tol=1e-11, restart=30, max_iter=3000, precision=precision)
    for f, op in enumerate(ops):
        Xb, rb = op.solve_batched(B[2 * f:2 * f + 2].clone(), tol=1e-11, restart=30, max_iter=3000,
                                  precision=precision)
        for k, J in enumerate(Js):
            r = 2 * f + k
            print(f"omega {OMEGAS[f]}: multifreq {reps[r].iters} iterations, single-operator batch {rb[k].iters}")
            assert reps[r].converged and reps[r].relres <= 1e-11
            assert abs(reps[r].iters - rb[k].iters) <= 0.1 * rb[k].iters + 2
            s = S["sys"][f]
            xo = remove_v_mean(s, direct(s, s.rhs(J)))
            assert np.linalg.norm(X[r].cpu().numpy() - xo) <= 1e-9 * np.linalg.norm(xo)
            assert torch.linalg.norm(X[r] - Xb[k]).item() <= 1e-9 * torch.linalg.norm(Xb[k]).item()


def test_multifreq_single_operator_equals_batched():
    """One operator: the same groups as eddy_solve_batched, bit for bit."""
    from paper_1602_03207_amd import eddy
    S = setup()
    op = S["ops"][1]
    B = torch.stack([op.rhs_from_current(torch.from_numpy(J).cuda()) for J in S["Js"]])
    X, reps = eddy.solve_multifreq([op], B, [0, 0], tol=1e-11, restart=30, max_iter=3000, precision="mixed16")
    Xb, rb = op.solve_batched(B.clone(), tol=1e-11, restart=30, max_iter=3000, precision="mixed16")
    assert [r.iters for r in reps] == [r.iters for r in rb]
    assert torch.equal(X, Xb)


def test_multifreq_rejects_what_cannot_be_factored():
    from paper_1602_03207_amd import eddy
    S = setup()
    ops = S["ops"]
    B = torch.stack([ops[0].rhs_from_current(torch.from_numpy(S["Js"][0]).cuda())] * 2)
    with pytest.raises(eddy.EddyError, match="nondecreasing"):
        eddy.solve_multifreq(ops[:2], B, [1, 0], precision="mixed")
    with pytest.raises(eddy.EddyError, match="precision >= 1"):
        eddy.solve_multifreq(ops[:2], B, [0, 1], precision="fp64")
    other = eddy.Operator(S["M"], tau=1.0, block_size=64)
    other.assemble(S["nu"], 2.0 * S["sig"], OMEGAS[0])
    with pytest.raises(eddy.EddyError, match="materials"):
        eddy.solve_multifreq([ops[0], other], B, [0, 1], precision="mixed")
