"""MI355X (gfx950) tall & skinny matrix products: TSMTTSM C = A^T B and TSMM B = A C."""
