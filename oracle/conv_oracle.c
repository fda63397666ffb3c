/* placeholder: convolution oracle is added with the learned coarse correction */
int orc_conv_placeholder(void) { return 0; }
