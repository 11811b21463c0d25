"""The oracle's reductions are serial loops in node order and OpenMP only splits
element-wise loops, so a run on one thread and on several gives the same bits."""
import numpy as np

from paper_1507_07666_amd import inputs as I


def test_oracle_results_do_not_depend_on_thread_count(oracle_mod):
    O = oracle_mod
    system = I.ne_atom().scaled(14)
    system.dims = (14, 11, 9)
    keep = O.max_threads()
    out = []
    try:
        for t in (1, 3):
            O.set_threads(t)
            o = O.oracle_for(system)
            for _ in range(6):
                o.step()
            psi, rho = o.state()
            out.append((psi.copy(), rho.copy(), o.energies(converge_poisson=True).e_total, o.forces()))
    finally:
        O.set_threads(keep)
    assert np.array_equal(out[0][0], out[1][0]) and np.array_equal(out[0][1], out[1][1])
    assert out[0][2] == out[1][2]
    assert np.array_equal(out[0][3], out[1][3])
