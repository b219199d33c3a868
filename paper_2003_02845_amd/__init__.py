"""MI355X (gfx950) implementation of one time step of the locally implicit
Lax-Wendroff discrete-ordinate neutrino transport scheme of Chan & Mueller
(arXiv:2003.02845), behind the C ABI declared in include/btx.h."""
