"""Band pairs of the heterocorrelation workload whose asynchronous sign the
generator fixes (Noda's rule on Psi, Sec. 2 Eq. (disHTasyn) with the sign
reading of the Hilbert-Noda kernel, Eq. (HilbNoda)).

Band k of a set follows latent driver d_k with phase phi_d; a band whose
driver leads (larger phase, both in [0, pi]) gives Psi > 0 against a band
that lags.  That holds at the band centres where each band dominates its
own centre's dynamic signal (the four-decade spread of the base amplitudes
lets a strong neighbour's tail take over a weak band's centre otherwise),
and for phase differences away from 0 and pi.  The selection below uses
only the generator's parameters, never a correlation result.
"""
import numpy as np

DOMINANCE = 3.0     # own dynamic amplitude at the centre / that of all other bands
MIN_SIN = 0.3       # |sin(phi_1 - phi_2)| of a selected pair


def _dominance(meta):
    c, g, base, w = meta["centers"], meta["hwhm"], meta["base"], meta["weight"]
    x = np.round(c)
    # Lorentzian profiles (the workload's bands) at each centre, times the
    # dynamic amplitude base * 0.3 w (the 0.3 cancels in the ratio)
    A = g[None, :] ** 2 / ((x[:, None] - c[None, :]) ** 2 + g[None, :] ** 2) * (base * w)[None, :]
    own = np.diag(A).copy()
    return own / (A.sum(axis=1) - own)


def lag_sign_pairs(meta):
    """(rows, cols, expected sign) at the selected band-centre pairs of
    synth.workload_hetero's meta."""
    m1, m2, ph = meta["set1"], meta["set2"], meta["driver_phase"]
    c1 = np.round(m1["centers"]).astype(np.int64)
    c2 = np.round(m2["centers"]).astype(np.int64)
    k, l = np.meshgrid(np.arange(len(c1)), np.arange(len(c2)), indexing="ij")
    k, l = k.ravel(), l.ravel()
    s = np.sin(ph[m1["driver"][k]] - ph[m2["driver"][l]])
    sel = ((_dominance(m1) > DOMINANCE)[k] & (_dominance(m2) > DOMINANCE)[l]
           & (np.abs(s) > MIN_SIN))
    return c1[k[sel]], c2[l[sel]], np.sign(s[sel])
