"""Second-order Trotter-Suzuki solver for AMD MI355X (gfx950)."""
