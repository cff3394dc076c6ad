"""MI355X (gfx950) implementation of the R factor of a tall-skinny QR by
Householder TSQR (Langou, arXiv:1002.4250)."""
