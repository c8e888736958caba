"""Test inputs, with their expected branches, on which the two deflation
tests of Sec. 1.1 and the h guard decide differently.  Used by the oracle
pins, the oracle mutation check and the GPU parity tests."""
import numpy as np

# a12 = 0, so the arrow is read off directly:
# alpha = (a11, a22), beta = (a13, a23), gamma = a33.  The tests are stated
# with |e| = |alpha beta1 beta2| / h^2 (alpha = alpha1 - alpha2) and
#   EISPACK:     |e| <= eps (|d1| + |d2|)
#   simplified:  |e| <= eps |alpha1 + alpha2|.
# D1: alpha = (1, -1), beta = (1e-17, 1), gamma = 0.25.  h = 1, |e| = 2e-17,
#     |d1| + |d2| = 2: the EISPACK test deflates (bound 2 eps = 4.4e-16); the
#     simplified bound is eps * 0 = 0, so that test does not.
# D2: alpha = (1, 0.5), beta = (1e-20, 1e-20), gamma = 0.25.  h = 1.4e-20 is
#     below eps (|alpha1| + |alpha2| + |gamma|) = 3.9e-16: diagonal under the
#     guard.  Without it (only h == 0 is diagonal) neither test deflates:
#     |e| = 0.25 against bounds of about 3.3e-16.
DEFLATION_CASES = np.array([[1.0, 0.0, 1e-17, -1.0, 1.0, 0.25],
                            [1.0, 0.0, 1e-20, 0.5, 1e-20, 0.25]])
# branch per flag combination (0, SIMPLIFIED, NO_H_GUARD, both): 2 diagonal,
# 3 deflated, 4 reduced
DEFLATION_BRANCHES = {0: [3, 2], 1: [4, 2], 2: [3, 4], 3: [4, 4]}
