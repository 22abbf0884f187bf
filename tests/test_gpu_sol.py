"""Per-stage getters of the solution object: filled from a batch instance
and from a server request, each stage block equals the matching slice of
the whole-vector result (user layout: per stage [box u, box x, general])."""
import time

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from paper_2003_02547_amd import binding as B  # noqa: E402
from paper_2003_02547_amd import workloads as W  # noqa: E402


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU visible")
    B.lib()


def check_stagewise(qp, sol_obj, whole):
    ou = ox = op = oc = 0
    for n in range(qp.N + 1):
        nu, nx = qp.nu[n], qp.nx[n]
        nbu, nbx, ng = qp.nbu[n], qp.nbx[n], qp.ng[n]
        assert np.array_equal(sol_obj.get("u", n, nu), whole["u"][ou:ou + nu])
        assert np.array_equal(sol_obj.get("x", n, nx), whole["x"][ox:ox + nx])
        if n < qp.N:
            m = qp.nx[n + 1]
            assert np.array_equal(sol_obj.get("pi", n, m), whole["pi"][op:op + m])
            op += m
        for pre, key in (("lam", "lam_"), ("t", "t_")):
            for side, vec in (("lb", whole[key + "l"]), ("ub", whole[key + "u"])):
                assert np.array_equal(sol_obj.get(f"{pre}_{side}_u", n, nbu), vec[oc:oc + nbu])
                assert np.array_equal(sol_obj.get(f"{pre}_{side}_x", n, nbx), vec[oc + nbu:oc + nbu + nbx])
            assert np.array_equal(sol_obj.get(f"{pre}_lg", n, ng), whole[key + "l"][oc + nbu + nbx:oc + nbu + nbx + ng])
            assert np.array_equal(sol_obj.get(f"{pre}_ug", n, ng), whole[key + "u"][oc + nbu + nbx:oc + nbu + nbx + ng])
        ou += nu
        ox += nx
        oc += nbu + nbx + ng


def test_sol_object_from_batch_and_server():
    rng = np.random.default_rng(21)
    qps = [W.random_tiny(rng, 4, ng_max=2) for _ in range(3)] + [W.mass_spring_chain4(2)]
    b = B.Batch(qps).load().solve().fetch().sync()
    for i, qp in enumerate(qps):
        s = B.Sol(B.Dims.of(qp)).fill_from_batch(b, i)
        check_stagewise(qp, s, b.solution(i))
        st = b.stat(i)
        assert np.array_equal(s.norms(), np.array(st.res[:]))
    # a mismatching dims object is refused
    other = B.Sol(B.Dims.of(qps[3]))
    with pytest.raises(B.OqpError):
        other.fill_from_batch(b, 0)
    srv = B.Server(B.default_arg(), dev_bytes=64 << 20, nstreams=2)
    try:
        p = B.Packed(qps[3], pinned=True)
        t = srv.submit(p)
        deadline = time.time() + 30
        while srv.poll(t) is None:
            assert time.time() < deadline
            srv.progress()
        s = B.Sol(B.Dims.of(qps[3])).fill_from_server(srv, t)
        check_stagewise(qps[3], s, srv.solution(t))
        srv.release(t)
    finally:
        srv.close()
