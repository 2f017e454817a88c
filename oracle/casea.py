"""Known-spectrum Hermitian J-symmetric matrices (the Case A recipe, Sec. 4.1).

Test infrastructure only (see the package docstring).  The recipe is an input
generator, so it lives with the other seeded inputs
(paper_2001_07428_amd.inputs.known_spectrum) and is re-exported here.

A = U diag(Lambda, Lambda) U^H with U = [[X1, -X2^*], [X2, X1^*]]
(eq. diagblockform), i.e. U = [X, J X^*] with X = [X1; X2].
"""
from paper_2001_07428_amd.inputs import known_spectrum  # noqa: F401
