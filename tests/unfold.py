"""Unfolding of a double-layered torus with one flipped boundary into the
periodic lattice of doubled extent (a test helper: index arithmetic only)."""
import numpy as np


def doubled_torus_map(L, mu):
    """Site map of the double-layered torus whose only flipped boundary is
    that of direction mu onto the periodic lattice with extent 2 L_mu: site
    (layer, x) goes to x' with x'_mu = x_mu + layer L_mu."""
    L2 = list(L)
    L2[mu] *= 2
    V = int(np.prod(L))
    stride = [int(np.prod(L[:m])) for m in range(4)]
    stride2 = [int(np.prod(L2[:m])) for m in range(4)]
    out = np.empty(2 * V, dtype=np.int64)
    for layer in range(2):
        for lex in range(V):
            x = [(lex // stride[m]) % L[m] for m in range(4)]
            x[mu] += layer * L[mu]
            out[layer * V + lex] = sum(x[m] * stride2[m] for m in range(4))
    return tuple(L2), out


def unfold_links(links, site):
    """Links (4 per site, canonical (n_links, 18) layout) moved to the unfolded site labels."""
    out = np.empty_like(links)
    for s in range(len(site)):
        out[4 * site[s]:4 * site[s] + 4] = links[4 * s:4 * s + 4]
    return out
