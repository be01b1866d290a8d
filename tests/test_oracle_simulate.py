"""End-to-end pin of the oracle: the ensemble covariance of pixels equals the simulator's
exact closed form sum_ab w_ia w_jb xi_lattice(x_a - x_b), with xi_lattice the inverse DFT
of P_box (eq. pboxxi)."""
import numpy as np

from oracle import gather, simulate, spectrum
from paper_2507_15703_amd import workloads


def test_pixel_covariance_closed_form():
    N, L, r = 8, 1.0, 0.3
    k, p = workloads.powerlaw_cutoff_table(N, L, kc_modes=2)
    dirs = np.array([[0, 0, 1.0], [0.6, 0, 0.8], [0, 0.6, 0.8], [-0.48, 0.6, 0.64]])
    dirs /= np.linalg.norm(dirs, axis=1, keepdims=True)
    for interp in (gather.TRILINEAR, gather.TRICUBIC):
        maps = np.array([simulate.simulate(N, L, 1000 + s, r, dirs, k, p, interp)[0] for s in range(1500)])
        emp = maps.T @ maps / maps.shape[0]
        # closed form
        pb = spectrum.p_box_table(N, L, k, p)
        f = np.arange(N)
        f = np.minimum(f, N - f)
        m = f[:, None, None] ** 2 + f[None, :, None] ** 2 + f[None, None, :] ** 2
        xi = np.real(np.fft.ifftn(pb[m])) * N**3
        idx, w = gather.stencil(N, L, r, dirs, interp)
        K = idx.shape[2]
        nodes, wts = [], []
        for i in range(len(dirs)):
            g = np.stack(np.meshgrid(*[idx[i, d] for d in range(3)], indexing="ij"), -1).reshape(-1, 3)
            ww = np.einsum("a,b,c->abc", w[i, 0], w[i, 1], w[i, 2]).reshape(-1)
            nodes.append(g)
            wts.append(ww)
        C = np.zeros((len(dirs), len(dirs)))
        for i in range(len(dirs)):
            for j in range(len(dirs)):
                d = (nodes[i][:, None, :] - nodes[j][None, :, :]) % N
                C[i, j] = wts[i] @ xi[d[..., 0], d[..., 1], d[..., 2]] @ wts[j]
        n = maps.shape[0]
        sd = np.sqrt((np.outer(np.diag(C), np.diag(C)) + C**2) / n)
        assert np.all(np.abs(emp - C) < 5 * sd), (interp, emp, C)
