"""Post-processing: B = curl A and the L2 flux-density error (oracle).

TEST INFRASTRUCTURE ONLY.

Section 4 measures eps_B = sqrt(sum_k ||B_ana - B_num||^2_{L2(Omega^(k))}).
Here the integrals use Gauss-Legendre with p+1 points per direction per
element (a reading; the paper does not state its rule), summed over patches
(which sums over subdomains).  The relative form divides by ||B_ref||.
"""
from __future__ import annotations

import numpy as np


def b_at_quadrature(space, a, ed=None):
    """Yield (points, |det| w, B) per patch for global coefficients a."""
    if ed is None:
        ed = space.element_data(0)
    for pidx in range(int(np.prod(space.P))):
        x, wdet, curl, _ = space.physical(pidx, ed)
        g = space.patch_local_edges(pidx)
        ae = a[g][ed["loc"]]  # (E, nf)
        B = np.einsum("eqaf,ef->eqa", curl, ae)
        yield x, wdet, B


def b_error(space, a, b_ref=None, a_ref=None):
    """(absolute, relative) L2 error of curl A_h against a field or another vector."""
    ed = space.element_data(0)
    num = 0.0
    den = 0.0
    if a_ref is not None:
        it_ref = b_at_quadrature(space, a_ref, ed)
    for x, wdet, B in b_at_quadrature(space, a, ed):
        if a_ref is not None:
            _, _, Br = next(it_ref)
        else:
            Br = b_ref(x.reshape(-1, 3)).reshape(B.shape)
        num += float(np.sum(wdet[:, :, None] * (B - Br) ** 2))
        den += float(np.sum(wdet[:, :, None] * Br ** 2))
    return np.sqrt(num), (np.sqrt(num / den) if den > 0 else np.sqrt(num))
